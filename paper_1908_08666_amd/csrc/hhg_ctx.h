// Handle definition and host helpers shared by the library's translation units.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "hhg_internal.h"

struct hhg_ctx {
  int n_macro = 0;
  int coupling = HHG_CONFORMING;
  int dirichlet = HHG_DIRICHLET_OUTER;
  hhg_op_desc op{};
  int max_level = 0;
  int64_t n_nodes = 0;
  int64_t n_unknown = 0;
  std::vector<double> verts;                 // [n_macro][4][3]
  std::vector<hhg::MacroInfo> minfo;         // host copy
  std::vector<uint8_t> flags;                // per slot: bit0 Dirichlet, bit1 owner, bit2 boundary,
                                             // bit3 node has copies in other macros
  std::vector<hhg::StencilConst<double>> sc64;
  std::vector<hhg::ElemConst<double>> ec64;
  std::vector<hhg::StrainConst> stc;
  std::vector<hhg::WorkItem> work;
  std::vector<int32_t> bijk;                 // non-Dirichlet boundary slots, packed (i,j,k)
  std::vector<int32_t> bblk;                 // macro of each boundary-row block
  std::vector<hhg::FaceTile> ftile;          // tiles of face-interior rows (non-Dirichlet faces)
  std::vector<int64_t> dslot;                // Dirichlet slots (rows written as zero)
  std::vector<int64_t> bnd;                  // every macro-boundary slot (flag bit 2)
  std::vector<int64_t> grp_ptr, grp_slot;    // non-Dirichlet copy groups
  std::vector<int64_t> agrp_ptr, agrp_slot;  // all copy groups
  int wl_max = 0;                            // LDS window entries per plane
  int planes_per_item = 0;                   // slab depth of every level (HHG_PLANES_PER_ITEM); 0: by level
  int slab_by_level[hhg::MAX_LEVEL + 1] = {};  // tuned slab depth per level (0: default)
  int persist_blocks = 0;                    // 0: one workgroup per item; else resident grid size
  int chunk = 256;                           // positions per interior work item
  bool serial_apply = false;                 // boundary rows on the caller's stream too
  bool on_device = false;                    // tables uploaded (first device call)
  int device = -1;

  // device copies
  hhg::MacroInfo *d_minfo = nullptr;
  hhg::StencilConst<double> *d_sc64 = nullptr;
  hhg::StencilConst<float> *d_sc32 = nullptr;
  hhg::ElemConst<double> *d_ec64 = nullptr;
  hhg::ElemConst<float> *d_ec32 = nullptr;
  hhg::WorkItem *d_work = nullptr;
  int n_work = 0;
  int32_t *d_bijk = nullptr;
  int32_t *d_bblk = nullptr;
  hhg::FaceTile *d_ftile = nullptr;
  int64_t *d_dslot = nullptr;
  int64_t *d_bnd = nullptr;
  int64_t n_bnd = 0;
  int64_t *d_grp_ptr = nullptr;              // interface copy groups (>= 2 copies)
  int64_t *d_grp_slot = nullptr;
  int64_t n_grp = 0;
  int64_t *d_agrp_ptr = nullptr;             // all copy groups (Dirichlet ones too)
  int64_t *d_agrp_slot = nullptr;
  int64_t n_agrp = 0;
  hhg::StrainConst *d_stc = nullptr;
  // strain-rate fit on macro-boundary nodes (built at the first viscosity
  // call): per distinct node its patch (slots and gradient weights [3]) and
  // the slots of its copies
  double *d_dotpart = nullptr;               // partial sums of the apply with (x, A x)
  int64_t dotpart_cap = 0;                   // their capacity (in partial sums)
  bool lsq_built = false;
  int64_t n_lsq = 0, n_lsq_affine = 0;
  int64_t *d_lsq_ptr = nullptr, *d_lsq_slot = nullptr;
  double *d_lsq_w = nullptr;
  int64_t *d_lsq_optr = nullptr, *d_lsq_oslot = nullptr;
  uint8_t *d_flags = nullptr;
  hipStream_t side = nullptr;                // macro-boundary rows run here
  hipStream_t solve_stream = nullptr;        // solvers run (and capture graphs) here
  void *h_state = nullptr;                   // pinned host mirror of the solver state
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  hhg_mlp model = nullptr;                   // learned smoother (not owned)

  // captured applies (hhg_graph_*): id -> executable graph
  struct GraphRec {
    int32_t id;
    hipGraphExec_t exec;
  };
  std::vector<GraphRec> graphs;
  int32_t next_graph_id = 1;

  // kernel timing (hhg_profile_*)
  struct ProfRec {
    int kid;
    hipEvent_t a, b;
  };
  bool prof_on = false;
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[HHG_K_COUNT] = {};
  int64_t prof_n[HHG_K_COUNT] = {};
};

namespace hhg {
int ensure_device(hhg_ctx *h);
// Interior work list over the given macros: slabs of slab[level] planes (or
// the default depth), 256-position chunks, interleaved so that item q runs on
// XCD q % NXCD with each XCD holding a contiguous stretch of the natural
// (macro, plane range, chunk) order.  Also returns the LDS window length.
void build_work(const hhg_ctx *h, const std::vector<int> &macros, const int *slab,
                std::vector<WorkItem> &out, int &wl_max);
void free_graphs(hhg_ctx *h);
// Default slab depth (planes per interior work item) of a level: deep slabs
// spread each item's start-up (three planes loaded before the first row) on
// the large levels; shallow ones give the small levels more items.
// Slab depth (planes per interior work item) of a level: HHG_PLANES_PER_ITEM
// when set, else 5 planes from level 7 up and 3 below.  SLAB_BALANCED asks
// build_work for segments of equal cost instead (every chunk column cut
// into about one segment per resident workgroup).
constexpr int SLAB_BALANCED = -1;
inline int default_slab(const hhg_ctx *h, int level) {
  if (h->planes_per_item > 0) return h->planes_per_item;
  return level >= 7 ? 5 : 3;
}

// Brackets one kernel launch with events when profiling is enabled.
class ProfScope {
 public:
  ProfScope(hhg_ctx *h, int kid, hipStream_t st);
  ~ProfScope();

 private:
  hhg_ctx *h_;
  int kid_;
  hipStream_t st_;
  hipEvent_t a_ = nullptr;
};
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
}  // namespace hhg

#define HHG_HIP(call)                                      \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hhg::hip_fail(e_, #call); \
  } while (0)
