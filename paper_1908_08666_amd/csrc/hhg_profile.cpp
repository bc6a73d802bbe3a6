// Event-based kernel timing of the library's own launches (tracing aid).
#include "hhg_ctx.h"

namespace hhg {

static hipEvent_t take_event(hhg_ctx *h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(hhg_ctx *h, int kid, hipStream_t st) : h_(h), kid_(kid), st_(st) {
  if (!h_->prof_on) return;
  a_ = take_event(h_);
  if (a_ && hipEventRecord(a_, st_) != hipSuccess) a_ = nullptr;
}

ProfScope::~ProfScope() {
  if (!h_->prof_on || !a_) return;
  hipEvent_t b = take_event(h_);
  if (!b || hipEventRecord(b, st_) != hipSuccess) return;
  h_->prof_pending.push_back({kid_, a_, b});
}

static int drain(hhg_ctx *h) {
  for (auto &r : h->prof_pending) {
    HHG_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    HHG_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    h->prof_ms[r.kid] += ms;
    h->prof_n[r.kid] += 1;
    h->ev_pool.push_back(r.a);
    h->ev_pool.push_back(r.b);
  }
  h->prof_pending.clear();
  return HHG_OK;
}

}  // namespace hhg

extern "C" {

int hhg_profile_enable(hhg_handle h, int32_t on) {
  if (!h) return hhg::fail(HHG_EINVAL, "null handle");
  int rc = hhg::drain(h);
  if (rc) return rc;
  for (int q = 0; q < HHG_K_COUNT; ++q) {
    h->prof_ms[q] = 0.0;
    h->prof_n[q] = 0;
  }
  h->prof_on = on != 0;
  return HHG_OK;
}

int hhg_profile_read(hhg_handle h, int32_t kernel_id, int64_t *launches, double *total_ms) {
  if (!h) return hhg::fail(HHG_EINVAL, "null handle");
  if (kernel_id < 0 || kernel_id >= HHG_K_COUNT) return hhg::fail(HHG_EINVAL, "bad kernel id");
  int rc = hhg::drain(h);
  if (rc) return rc;
  if (launches) *launches = h->prof_n[kernel_id];
  if (total_ms) *total_ms = h->prof_ms[kernel_id];
  return HHG_OK;
}

}  // extern "C"
