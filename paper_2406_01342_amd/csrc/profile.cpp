// Per-kernel instrumentation of a plan: HIP events around each launch on its
// own stream, resolved lazily, accumulated per kernel name.
#include <cstring>

#include "common.h"

namespace pc {

static hipEvent_t take_event(pc_plan* p) {
  if (!p->prof.pool.empty()) {
    hipEvent_t e = p->prof.pool.back();
    p->prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  PC_HIP(hipEventCreate(&e));
  return e;
}

ProfScope::ProfScope(pc_plan* plan, hipStream_t stream, const char* kname, double b, double w)
    : p(plan), s(stream), name(kname), bytes(b), work(w) {
  if (!p || !p->prof.on) return;
  a = take_event(p);
  PC_HIP(hipEventRecord(a, s));
}

ProfScope::~ProfScope() {
  if (!a) return;
  hipEvent_t b = nullptr;
  try {
    b = take_event(p);
  } catch (...) {
    return;
  }
  if (hipEventRecord(b, s) != hipSuccess) return;
  auto& st = p->prof.stats;
  int idx = -1;
  for (size_t i = 0; i < st.size(); ++i)
    if (st[i].name == name) {
      idx = (int)i;
      break;
    }
  if (idx < 0) {
    st.push_back(KStat{});
    st.back().name = name;
    idx = (int)st.size() - 1;
  }
  st[idx].launches += 1;
  st[idx].bytes += bytes;
  st[idx].work += work;
  p->prof.pending.push_back({idx, a, b});
  if (p->prof.pending.size() >= 4096) {
    try {
      prof_flush(p);
    } catch (...) {
    }
  }
}

void prof_flush(pc_plan* p) {
  for (auto& q : p->prof.pending) {
    PC_HIP(hipEventSynchronize(q.b));
    float ms = 0;
    PC_HIP(hipEventElapsedTime(&ms, q.a, q.b));
    p->prof.stats[q.idx].ms += ms;
    p->prof.pool.push_back(q.a);
    p->prof.pool.push_back(q.b);
  }
  p->prof.pending.clear();
}

void prof_reset(pc_plan* p) {
  prof_flush(p);
  p->prof.stats.clear();
}

void prof_release(pc_plan* p) {
  for (auto& q : p->prof.pending) {
    (void)hipEventDestroy(q.a);
    (void)hipEventDestroy(q.b);
  }
  p->prof.pending.clear();
  for (auto e : p->prof.pool) (void)hipEventDestroy(e);
  p->prof.pool.clear();
}

}  // namespace pc

using namespace pc;

template <typename F>
static pc_status prof_guard(const char* fn, F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_last_error(std::string(fn) + ": " + e.what());
    return e.status;
  }
}

extern "C" {

PC_API pc_status pc_plan_profile(pc_plan* p, int32_t enable) {
  return prof_guard("pc_plan_profile", [&] {
    PC_REQUIRE(p != nullptr, "plan is NULL");
    PC_HIP(hipSetDevice(p->device));
    prof_reset(p);
    p->prof.on = enable != 0;
    return PC_OK;
  });
}

PC_API pc_status pc_plan_kernel_stat(pc_plan* p, int32_t index, pc_kernel_stat* out) {
  return prof_guard("pc_plan_kernel_stat", [&] {
    PC_REQUIRE(p != nullptr && out != nullptr, "NULL argument");
    PC_HIP(hipSetDevice(p->device));
    prof_flush(p);
    PC_REQUIRE(index >= 0 && index < (int32_t)p->prof.stats.size(), "index out of range");
    const KStat& k = p->prof.stats[index];
    std::memset(out, 0, sizeof(*out));
    std::strncpy(out->name, k.name.c_str(), sizeof(out->name) - 1);
    out->launches = k.launches;
    out->ms = k.ms;
    out->bytes = k.bytes;
    out->work = k.work;
    return PC_OK;
  });
}

PC_API int32_t pc_plan_kernel_stat_count(pc_plan* p) {
  return p ? (int32_t)p->prof.stats.size() : 0;
}

}  // extern "C"
