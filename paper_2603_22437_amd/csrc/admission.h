// Admission by device-memory footprint with least-recently-used residency of
// per-tenant evaluation keys.  Host logic only (no HIP), shared by the serving
// runtime and its CPU tests.
//
// Every tenant has a key footprint.  A request is admitted when its tenant's
// keys are resident, or can be made resident, and the request's own working
// set fits: the resident keys plus the working sets of admitted requests
// never exceed the budget.  To make room, the policy evicts resident tenants
// with no admitted request, least recently used first.  It never evicts a
// tenant whose keys an admitted request still uses.
#pragma once

#include <algorithm>
#include <cstdint>
#include <map>
#include <vector>

namespace hck {

class Residency {
 public:
  enum Decision { kAdmit, kWait, kReject };

  explicit Residency(uint64_t budget) : budget_(budget) {}

  // registers (or re-sizes, while not resident) a tenant's key footprint
  bool add_tenant(uint32_t t, uint64_t key_bytes) {
    auto it = ts_.find(t);
    if (it != ts_.end() && (it->second.resident || it->second.active)) return false;
    ts_[t] = Entry{key_bytes, false, 0, 0};
    return true;
  }

  // Decides on one request of tenant t with `extra` bytes of working set.
  // kAdmit: the request is accounted; `evict` lists the tenants whose keys
  // must be released first and `load` says whether t's keys must be loaded.
  // kWait: not now (the budget is held by admitted requests).  kReject: never
  // (the request alone exceeds the budget, or t is unknown).
  Decision admit(uint32_t t, uint64_t extra, std::vector<uint32_t> &evict, bool &load) {
    evict.clear();
    load = false;
    auto it = ts_.find(t);
    if (it == ts_.end()) return kReject;
    Entry &e = it->second;
    const uint64_t need = extra + (e.resident ? 0 : e.bytes);
    if (extra + e.bytes > budget_) return kReject;
    if (used_ + need > budget_) {
      // least recently used idle tenants first
      std::vector<std::pair<uint64_t, uint32_t>> idle;
      for (auto &kv : ts_)
        if (kv.first != t && kv.second.resident && kv.second.active == 0)
          idle.push_back({kv.second.last, kv.first});
      std::sort(idle.begin(), idle.end());
      uint64_t freed = 0;
      for (auto &c : idle) {
        if (used_ - freed + need <= budget_) break;
        evict.push_back(c.second);
        freed += ts_[c.second].bytes;
      }
      if (used_ - freed + need > budget_) {
        evict.clear();
        return kWait;
      }
      for (uint32_t v : evict) {
        ts_[v].resident = false;
        used_ -= ts_[v].bytes;
      }
    }
    if (!e.resident) {
      e.resident = true;
      load = true;
      used_ += e.bytes;
    }
    used_ += extra;
    e.active++;
    e.last = ++clock_;
    return kAdmit;
  }

  // a request of t that was admitted with `extra` bytes has finished
  void release(uint32_t t, uint64_t extra) {
    auto it = ts_.find(t);
    if (it == ts_.end() || it->second.active == 0) return;
    it->second.active--;
    used_ -= std::min(used_, extra);
  }

  // evicts one idle resident tenant (after its keys failed to load)
  bool evict(uint32_t t) {
    auto it = ts_.find(t);
    if (it == ts_.end() || !it->second.resident || it->second.active) return false;
    it->second.resident = false;
    used_ -= it->second.bytes;
    return true;
  }

  // evicts every idle resident tenant (teardown); returns them
  std::vector<uint32_t> evict_idle() {
    std::vector<uint32_t> out;
    for (auto &kv : ts_)
      if (kv.second.resident && kv.second.active == 0) {
        kv.second.resident = false;
        used_ -= kv.second.bytes;
        out.push_back(kv.first);
      }
    return out;
  }

  bool resident(uint32_t t) const {
    auto it = ts_.find(t);
    return it != ts_.end() && it->second.resident;
  }
  uint32_t active(uint32_t t) const {
    auto it = ts_.find(t);
    return it == ts_.end() ? 0 : it->second.active;
  }
  uint64_t used() const { return used_; }
  uint64_t budget() const { return budget_; }

 private:
  struct Entry {
    uint64_t bytes;
    bool resident;
    uint32_t active;
    uint64_t last;
  };
  std::map<uint32_t, Entry> ts_;
  uint64_t budget_, used_ = 0, clock_ = 0;
};

}  // namespace hck
