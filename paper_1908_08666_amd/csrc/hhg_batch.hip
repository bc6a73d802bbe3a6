// Batching support for many macros (or many independent problems of uneven
// level) in one interior launch:
//
//   hhg_autotune      times the interior kernel per level over candidate slab
//                     depths (planes per work item), then the whole list over
//                     candidate grids (one workgroup per item, or a persistent
//                     grid of resident workgroups), and keeps the fastest.
//   hhg_graph_*       captures a sequence of applies once in a HIP graph and
//                     replays it with one launch.
//
// Tuning changes only which workgroup computes which rows: every row is
// still computed by one thread with the same arithmetic, so results are
// bitwise identical for every configuration.
#include <algorithm>
#include <cstring>
#include <vector>

#include "hhg_device.h"

namespace hhg {

int apply_entry(hhg_ctx *h, int prec, int method, const void *f, const void *x, const void *k,
                void *y, void *stream);
int apply_internal(hhg_ctx *h, int prec, int method, const void *f, const void *x, const void *k,
                   void *y, hipStream_t st);

namespace {

int launch_rows(hhg_ctx *h, int prec, int method, const void *x, const void *k, void *y,
                hipStream_t st) {
  if (prec == HHG_F64)
    return method == METHOD_SCALED
               ? launch_interior_v<double, METHOD_SCALED, false>(h, (const double *)x,
                                                                 (const double *)k, nullptr,
                                                                 (double *)y, st)
               : launch_interior_v<double, METHOD_ONTHEFLY, false>(h, (const double *)x,
                                                                   (const double *)k, nullptr,
                                                                   (double *)y, st);
  return method == METHOD_SCALED
             ? launch_interior_v<float, METHOD_SCALED, false>(h, (const float *)x, (const float *)k,
                                                              nullptr, (float *)y, st)
             : launch_interior_v<float, METHOD_ONTHEFLY, false>(h, (const float *)x,
                                                                (const float *)k, nullptr,
                                                                (float *)y, st);
}

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Device copy of a work list, freed on scope exit unless released.
struct DevList {
  WorkItem *p = nullptr;
  ~DevList() {
    if (p) (void)hipFree(p);
  }
};

void destroy_graphs(hhg_ctx *h) {
  for (auto &g : h->graphs) (void)hipGraphExecDestroy(g.exec);
  h->graphs.clear();
}

int autotune_impl(hhg_ctx *h, int prec, int method, const void *x, const void *k, void *y,
                  int reps, hhg_tune_report *rep, hipStream_t st) {
  std::memset(rep, 0, sizeof(*rep));
  // levels present, ascending
  std::vector<int> levels;
  for (auto &mi : h->minfo) levels.push_back(mi.level);
  std::sort(levels.begin(), levels.end());
  levels.erase(std::unique(levels.begin(), levels.end()), levels.end());

  Events ev;
  HHG_HIP(hipEventCreate(&ev.a));
  HHG_HIP(hipEventCreate(&ev.b));
  const bool prof = h->prof_on;
  h->prof_on = false;
  WorkItem *const d_keep = h->d_work;
  const int n_keep = h->n_work;
  const int persist_keep = h->persist_blocks;
  auto restore = [&]() {
    h->d_work = d_keep;
    h->n_work = n_keep;
    h->persist_blocks = persist_keep;
    h->prof_on = prof;
  };
  // average duration of `reps` interior launches after one warm-up
  auto time_list = [&](double &ms) -> int {
    int rc = launch_rows(h, prec, method, x, k, y, st);
    if (rc) return rc;
    HHG_HIP(hipEventRecord(ev.a, st));
    for (int r = 0; r < reps; ++r)
      if ((rc = launch_rows(h, prec, method, x, k, y, st))) return rc;
    HHG_HIP(hipEventRecord(ev.b, st));
    HHG_HIP(hipEventSynchronize(ev.b));
    float t = 0.f;
    HHG_HIP(hipEventElapsedTime(&t, ev.a, ev.b));
    ms = t / reps;
    return HHG_OK;
  };
  auto upload_list = [&](const std::vector<WorkItem> &items, DevList &dl) -> int {
    if (dl.p) {
      HHG_HIP(hipFree(dl.p));
      dl.p = nullptr;
    }
    HHG_HIP(hipMalloc((void **)&dl.p, std::max<size_t>(1, items.size()) * sizeof(WorkItem)));
    HHG_HIP(hipMemcpy(dl.p, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    h->d_work = dl.p;
    h->n_work = (int)items.size();
    return HHG_OK;
  };

  int slab[MAX_LEVEL + 1] = {};
  int ncand = 0;
  std::vector<WorkItem> items;
  int wl = 0;
  for (size_t li = 0; li < levels.size(); ++li) {
    const int L = levels[li];
    std::vector<int> ms_of;
    int64_t rows = 0;
    for (int m = 0; m < h->n_macro; ++m)
      if (h->minfo[m].level == L) {
        ms_of.push_back(m);
        const int64_t n = h->minfo[m].n;
        rows += (n - 1) * (n - 2) * (n - 3) / 6;
      }
    rep->level[li] = L;
    rep->macros[li] = (int)ms_of.size();
    rep->rows[li] = rows;
    const int n = 1 << L;
    double best = 1e30;
    int best_q = default_slab(h, L);
    // candidates: balanced segments, then slabs of 1, 2, 4, ... planes
    for (int q = SLAB_BALANCED; q <= std::max(1, 2 * (n - 3)); q = q > 0 ? 2 * q : 1) {
      int tmp[MAX_LEVEL + 1] = {};
      tmp[L] = q;
      build_work(h, ms_of, tmp, items, wl);
      DevList dl;
      int rc = upload_list(items, dl);
      if (!rc) {
        h->persist_blocks = 0;
        double ms = 0.0;
        rc = time_list(ms);
        ++ncand;
        if (!rc && ms < best) {
          best = ms;
          best_q = q;
        }
      }
      h->d_work = d_keep;  // dl frees the temporary list
      h->n_work = n_keep;
      if (rc) {
        restore();
        return rc;
      }
    }
    slab[L] = best_q;
    rep->slab[li] = best_q;
    rep->ms[li] = best;
  }
  rep->n_levels = (int)levels.size();

  // whole list with the chosen slabs; then the grid
  std::vector<int> all(h->n_macro);
  for (int m = 0; m < h->n_macro; ++m) all[m] = m;
  build_work(h, all, slab, items, wl);
  DevList fin;
  int rc = upload_list(items, fin);
  if (rc) {
    restore();
    return rc;
  }
  int cus = 0;
  HHG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
  const int grids[] = {0, cus, 2 * cus, 3 * cus, 4 * cus};
  double best = 1e30;
  int best_g = 0;
  for (int g : grids) {
    if (g % NXCD) continue;  // keep item q on XCD q % NXCD
    h->persist_blocks = g;
    double ms = 0.0;
    if ((rc = time_list(ms))) {
      h->d_work = d_keep;
      h->n_work = n_keep;
      restore();
      return rc;
    }
    ++ncand;
    if (ms < best) {
      best = ms;
      best_g = g;
    }
  }
  // adopt: the old list is freed, graphs captured with it are dropped
  destroy_graphs(h);
  if (d_keep) (void)hipFree(d_keep);
  h->d_work = fin.p;
  fin.p = nullptr;
  h->n_work = (int)items.size();
  h->work = items;
  h->persist_blocks = best_g;
  h->prof_on = prof;
  for (int L = 0; L <= MAX_LEVEL; ++L) h->slab_by_level[L] = slab[L];
  rep->persist_blocks = best_g;
  rep->ms_total = best;
  rep->candidates = ncand;
  // leave y = A x under the tuned configuration
  rc = apply_internal(h, prec, method, nullptr, x, k, y, st);
  if (rc) return rc;
  HHG_HIP(hipStreamSynchronize(st));
  return HHG_OK;
}

}  // namespace

int autotune_entry(hhg_ctx *h, int prec, int method, const void *x, const void *k, void *y,
                   int reps, hhg_tune_report *rep, void *stream) {
  if (!rep) return fail(HHG_EINVAL, "null report");
  if (reps < 1 || reps > 1000) return fail(HHG_EINVAL, "reps must lie in 1..1000");
  // argument checks, device upload and a warm-up: one ordinary apply
  int rc = apply_entry(h, prec, method, nullptr, x, k, y, stream);
  if (rc) return rc;
  return autotune_impl(h, prec, method, x, k, y, reps, rep, (hipStream_t)stream);
}

int set_tuning(hhg_ctx *h, const hhg_tune_report *t) {
  if (!t) return fail(HHG_EINVAL, "null tuning record");
  if (t->n_levels < 0 || t->n_levels > 8) return fail(HHG_EINVAL, "n_levels must lie in 0..8");
  if (t->persist_blocks != 0 &&
      (t->persist_blocks < NXCD || t->persist_blocks > 65536 || t->persist_blocks % NXCD))
    return fail(HHG_EINVAL, "persist_blocks must be 0 or a multiple of 8 in 8..65536");
  int slab[MAX_LEVEL + 1] = {};
  for (int q = 0; q < t->n_levels; ++q) {
    const int L = t->level[q];
    if (L < MIN_LEVEL || L > MAX_LEVEL) return fail(HHG_EINVAL, "level outside 2..8");
    if (t->slab[q] < SLAB_BALANCED || t->slab[q] > 1024)
      return fail(HHG_EINVAL, "slab outside -1..1024");
    slab[L] = t->slab[q];
  }
  int rc = ensure_device(h);
  if (rc) return rc;
  std::vector<int> all(h->n_macro);
  for (int m = 0; m < h->n_macro; ++m) all[m] = m;
  std::vector<WorkItem> items;
  int wl = 0;
  build_work(h, all, slab, items, wl);
  DevList dl;
  HHG_HIP(hipMalloc((void **)&dl.p, std::max<size_t>(1, items.size()) * sizeof(WorkItem)));
  HHG_HIP(hipMemcpy(dl.p, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
  // launches already queued may still read the old list
  HHG_HIP(hipDeviceSynchronize());
  destroy_graphs(h);
  if (h->d_work) (void)hipFree(h->d_work);
  h->d_work = dl.p;
  dl.p = nullptr;
  h->n_work = (int)items.size();
  h->work = std::move(items);
  h->persist_blocks = t->persist_blocks;
  for (int L = 0; L <= MAX_LEVEL; ++L) h->slab_by_level[L] = slab[L];
  return HHG_OK;
}

int graph_create(hhg_ctx *h, int prec, int method, const void *x, const void *k, void *y,
                 int count, int32_t *id) {
  if (!id) return fail(HHG_EINVAL, "null graph id");
  if (count < 1 || count > 1024) return fail(HHG_EINVAL, "count must lie in 1..1024");
  // checks and device upload by one eager apply on the handle's own stream,
  // after all work already queued on the device (the inputs) has finished
  int rc = ensure_device(h);
  if (rc) return rc;
  HHG_HIP(hipDeviceSynchronize());
  hipStream_t st = h->solve_stream;
  if ((rc = apply_entry(h, prec, method, nullptr, x, k, y, st))) return rc;
  HHG_HIP(hipStreamSynchronize(st));
  const bool prof = h->prof_on;
  h->prof_on = false;  // no timing events inside a graph
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    h->prof_on = prof;
    return hip_fail(e, "hipStreamBeginCapture");
  }
  for (int r = 0; r < count && !rc; ++r) rc = apply_internal(h, prec, method, nullptr, x, k, y, st);
  e = hipStreamEndCapture(st, &graph);
  h->prof_on = prof;
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  *id = h->next_graph_id++;
  h->graphs.push_back({*id, exec});
  return HHG_OK;
}

int graph_launch(hhg_ctx *h, int32_t id, void *stream) {
  for (auto &g : h->graphs)
    if (g.id == id) {
      HHG_HIP(hipGraphLaunch(g.exec, (hipStream_t)stream));
      return HHG_OK;
    }
  return fail(HHG_EINVAL, "unknown graph id (never created, destroyed, or dropped by hhg_autotune)");
}

int graph_destroy(hhg_ctx *h, int32_t id) {
  for (size_t q = 0; q < h->graphs.size(); ++q)
    if (h->graphs[q].id == id) {
      (void)hipGraphExecDestroy(h->graphs[q].exec);
      h->graphs.erase(h->graphs.begin() + q);
      return HHG_OK;
    }
  return fail(HHG_EINVAL, "unknown graph id");
}

void free_graphs(hhg_ctx *h) { destroy_graphs(h); }

}  // namespace hhg

extern "C" {

int hhg_autotune(hhg_handle h, int32_t prec, int32_t method, const void *x, const void *k, void *y,
                 int32_t reps, hhg_tune_report *report, void *stream) {
  return hhg::autotune_entry(h, prec, method, x, k, y, reps, report, stream);
}

int hhg_set_tuning(hhg_handle h, const hhg_tune_report *tuning) {
  if (!h) return hhg::fail(HHG_EINVAL, "null handle");
  return hhg::set_tuning(h, tuning);
}

int hhg_graph_create(hhg_handle h, int32_t prec, int32_t method, const void *x, const void *k,
                     void *y, int32_t count, int32_t *graph_id) {
  if (!h) return hhg::fail(HHG_EINVAL, "null handle");
  return hhg::graph_create(h, prec, method, x, k, y, count, graph_id);
}

int hhg_graph_launch(hhg_handle h, int32_t graph_id, void *stream) {
  if (!h) return hhg::fail(HHG_EINVAL, "null handle");
  return hhg::graph_launch(h, graph_id, stream);
}

int hhg_graph_destroy(hhg_handle h, int32_t graph_id) {
  if (!h) return hhg::fail(HHG_EINVAL, "null handle");
  return hhg::graph_destroy(h, graph_id);
}

}  // extern "C"
