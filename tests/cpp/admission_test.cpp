// CPU checks of the serving runtime's admission policy (Residency): budget
// accounting, least-recently-used eviction of idle tenants only, waiting
// while admitted work holds the budget, rejection of requests that can never
// fit.  Exits 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "admission.h"

using hck::Residency;

static int failures = 0;
#define CHECK(cond)                                                  \
  do {                                                               \
    if (!(cond)) {                                                   \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #cond); \
      failures++;                                                    \
    }                                                                \
  } while (0)

int main() {
  // budget 100: tenants of 40 bytes of keys, requests of 5
  Residency r(100);
  for (uint32_t t = 0; t < 4; t++) CHECK(r.add_tenant(t, 40));
  std::vector<uint32_t> ev;
  bool load = false;
  CHECK(r.admit(0, 5, ev, load) == Residency::kAdmit && load && ev.empty());
  CHECK(r.used() == 45);
  // the same tenant again: no load
  CHECK(r.admit(0, 5, ev, load) == Residency::kAdmit && !load);
  CHECK(r.used() == 50);
  CHECK(r.admit(1, 5, ev, load) == Residency::kAdmit && load && ev.empty());
  CHECK(r.used() == 95);
  // tenant 2 needs 45 more: 0 and 1 are active, so it waits
  CHECK(r.admit(2, 5, ev, load) == Residency::kWait && ev.empty());
  CHECK(r.used() == 95);
  // 1 finishes: now idle and evictable
  r.release(1, 5);
  CHECK(r.used() == 90 && r.active(1) == 0 && r.resident(1));
  CHECK(r.admit(2, 5, ev, load) == Residency::kAdmit && load);
  CHECK(ev.size() == 1 && ev[0] == 1 && !r.resident(1) && r.resident(2));
  CHECK(r.used() == 95);
  // least recently used first: finish everything, touch 0 last
  r.release(0, 5);
  r.release(0, 5);
  r.release(2, 5);
  CHECK(r.used() == 80);
  CHECK(r.admit(2, 5, ev, load) == Residency::kAdmit && !load);
  r.release(2, 5);
  CHECK(r.admit(0, 5, ev, load) == Residency::kAdmit && !load);
  r.release(0, 5);
  // 2 was used before 0, so loading 3 evicts 2
  CHECK(r.admit(3, 5, ev, load) == Residency::kAdmit && load);
  CHECK(ev.size() == 1 && ev[0] == 2);
  CHECK(r.resident(0) && r.resident(3) && !r.resident(2));
  CHECK(r.used() == 85);
  // a request that can never fit is rejected, an unknown tenant too
  Residency small(30);
  small.add_tenant(7, 40);
  CHECK(small.admit(7, 1, ev, load) == Residency::kReject && small.used() == 0);
  CHECK(small.admit(8, 1, ev, load) == Residency::kReject);
  // a failed key load is undone: release then evict
  Residency f(100);
  f.add_tenant(1, 60);
  CHECK(f.admit(1, 10, ev, load) == Residency::kAdmit && load);
  f.release(1, 10);
  CHECK(f.evict(1) && !f.resident(1) && f.used() == 0);
  // several evictions at once, in LRU order, never an active tenant
  Residency m(100);
  for (uint32_t t = 0; t < 5; t++) m.add_tenant(t, 20);
  for (uint32_t t = 0; t < 4; t++) {
    CHECK(m.admit(t, 0, ev, load) == Residency::kAdmit);
  }
  m.release(0, 0);
  m.release(2, 0);  // 1 and 3 stay active
  CHECK(m.used() == 80);
  m.add_tenant(9, 60);
  CHECK(m.admit(9, 0, ev, load) == Residency::kAdmit && load);
  CHECK(ev.size() == 2 && ev[0] == 0 && ev[1] == 2);
  CHECK(m.used() == 100 && m.resident(1) && m.resident(3));
  // a resident tenant cannot be re-sized, an idle unloaded one can
  CHECK(!m.add_tenant(9, 10));
  CHECK(m.add_tenant(0, 10));
  if (failures == 0) std::printf("admission: all checks passed\n");
  return failures ? 1 : 0;
}
