// Internal declarations of the mtspd library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <map>
#include <unordered_map>
#include <vector>

#include "../../include/mtspd.h"

namespace mts {

struct HipError {
  hipError_t err;
  const char *expr;
  const char *file;
  int line;
};
struct ArgError {
  std::string msg;
};
struct MemError {
  std::string msg;
};

#define MTS_HIP(expr)                                                   \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess) throw ::mts::HipError{e_, #expr, __FILE__, __LINE__}; \
  } while (0)

#define MTS_LAUNCH_CHECK() MTS_HIP(hipGetLastError())

// Device allocations of one solver: hipMalloc per allocation, or first-fit
// sub-allocation (256-byte aligned, freed extents coalesced) inside a
// caller-owned region that the solver never frees.
struct DeviceArena {
  std::vector<std::pair<void *, size_t>> blocks;
  size_t live = 0;  // bytes held now
  char *region = nullptr;
  size_t region_bytes = 0;
  std::map<size_t, size_t> free_ext, used_ext;  // offset -> size
  void use_region(void *base, size_t n) {
    region = static_cast<char *>(base);
    region_bytes = n & ~size_t(255);
    free_ext.clear();
    used_ext.clear();
    if (region_bytes) free_ext[0] = region_bytes;
  }
  template <class T>
  T *alloc(size_t n) {
    size_t b = sizeof(T) * (n ? n : 1);
    b = (b + 255) & ~size_t(255);
    void *p = nullptr;
    if (region) {
      auto it = free_ext.begin();
      while (it != free_ext.end() && it->second < b) ++it;
      if (it == free_ext.end())
        throw MemError{"caller arena of " + std::to_string(region_bytes) + " bytes is too small"};
      const size_t off = it->first, sz = it->second;
      free_ext.erase(it);
      if (sz > b) free_ext[off + b] = sz - b;
      used_ext[off] = b;
      p = region + off;
    } else {
      if (hipMalloc(&p, b) != hipSuccess) {
        (void)hipGetLastError();
        throw MemError{"hipMalloc of " + std::to_string(b) + " bytes failed"};
      }
      blocks.push_back({p, b});
    }
    live += b;
    return static_cast<T *>(p);
  }
  void release(void *p);
  void free_all();
};

constexpr int WAVE = 64;
constexpr int kSpareIters = 16;  // zero iterations appended to every sliced-ELL array

// Scalars of one problem, passed by value to kernels.
struct Params {
  int dim;
  int weight_kind;
  int kernel;
  int coupled;
  double delta, d2, V, VV, c0, lexp, scrit, K2;  // K2 = (1 + s_crit)^2
  double dtP, hdtP, hdt2P, dtF, hdtF, hdt2F;
  double o2lo[3], o2hi[3];
  double overlap;
  double rho;
  float K2m1f;  // (1 + s_crit)^2 - 1 in single precision (mixed-form stretch test)
};

// Sliced-ELL bond layout with L lanes per row: a slice is 64/L consecutive rows
// (one wavefront).  Slot k of local row j sits at
//   slot_off[slice] + (k / L) * 64 + j * L + k % L,
// so iteration t = k / L of the wavefront reads 64 consecutive slots.  Bond
// states are one 64-bit word per (slice, t), bit = lane, owned by the wavefront.
struct Sell {
  int64_t n_rows = 0, n_slices = 0, n_slots = 0, n_words = 0;
  int L = 1;
  int T = 0;                     // iterations per slice (same for every slice)
  int32_t *rows = nullptr;       // row -> node id
  int32_t *row_of = nullptr;     // node -> row (full layout in tile order; nullptr: identity)
  int32_t *width = nullptr;      // per slice, slots per row rounded up to a multiple of L
  int64_t *slot_off = nullptr;   // per slice, in slots (multiple of 64)
  int64_t *word_off = nullptr;   // per slice, in mask words
  int32_t *col = nullptr;        // n_slots
  uint64_t *mask = nullptr;      // n_words
  double *coef = nullptr;        // n_slots: w_ik c(|xi_ik|) V_i V_k (0 on padding)
  int32_t *slice_layer = nullptr; // link region: smallest h with a row within h horizons of a constraint
  float *coef32 = nullptr;       // mixed form: coef / m_i in single precision
  // full layout only: index and coefficient of each slot interleaved for the
  // bond pass, one load per slot (FP64: 3 dwords {col, coef}; mixed: 2 dwords
  // {col, coef32})
  uint32_t *slots = nullptr;
  // Neighbour staging (full layout): workgroup w runs slices
  // wg_start[w] .. wg_start[w + 1] - 1 (at most wg_waves, one spatial tile),
  // first copies the node records halo_ids[halo_off[w] .. halo_off[w + 1])
  // into LDS, and the offset field of its slot records points into that list.
  int32_t *halo_off = nullptr, *halo_ids = nullptr, *wg_start = nullptr;
  int64_t n_wg = 0;
  int32_t halo_max = 0;  // 0: no staging
  // Workgroups whose staged lists hold a row of workgroup w, or whose rows w's
  // list holds (a symmetric relation): dep_ids[dep_off[w] .. dep_off[w + 1]).
  // Workgroup w of a substep may start once these finished the previous one.
  int32_t *dep_off = nullptr, *dep_ids = nullptr;
  int32_t max_deps = 0;
  uint32_t *wg_flag = nullptr;  // per workgroup: the last substep it finished (epoch-numbered)
  int32_t wg_waves = 4;  // at most this many slices (wavefronts) per workgroup of the staged pass
  std::vector<int64_t> h_tile;  // host: spatial tile of each row (empty: rows not tiled)
  bool fp64_slots = false;      // slot records keep FP64 coefficients in the mixed form too
  bool pair_slots = false;      // mixed staged pass: one record per two iterations (16-bit list positions)
};

// Lanes per row: enough wavefronts to cover the chip, with as few lanes per row
// as that allows (fewer partial sums to combine); 3D rows are four times longer.
// `target` is the number of lanes of work to reach (0: the bond-pass default).
inline int pick_lanes(int64_t rows, int dim = 2, int64_t target = 0) {
  // 2D: two lanes per row on the 400x160 plate measured 5 % faster than four
  // (and one slower); the 1000x400 plate runs best at one
  if (target <= 0) target = dim == 3 ? ((int64_t)1 << 18) : (int64_t)128000;
  int L = 1;
  while (L < 8 && rows * L < target) L *= 2;
  return L;
}

struct Solver {
  mts_problem p{};
  std::vector<double> pos;   // host copy, node-major
  std::vector<double> cracks;
  int dim = 2;
  int64_t N = 0;
  hipStream_t stream = nullptr;
  int device = 0;                // HIP device current at create
  DeviceArena arena;
  Params prm{};
  int precision = MTS_FP64;
  bool breaking = true;
  int m = 1;
  bool unstable = false;
  bool wait_gave_up = false;     // a bounded wait of the subcycle kernel gave up (sticky)
  int64_t pd_steps = 0, macro_steps = 0, n_rebuilds = 0;
  int64_t n_intact0 = 0;  // intact bonds after setup (pre-crack cuts removed)
  std::vector<int64_t> h_node_tile;  // host: spatial tile of each node (empty: rows not tiled)
  double dt_bound_pd = 0.0;  // PD stability bound of the step

  // ---- PD ----
  double *x = nullptr;           // SoA dim*N
  float *xf = nullptr;           // SoA dim*N, positions minus the PD box origin (mixed)
  double *alpha = nullptr, *mass = nullptr, *P = nullptr;
  // Node records [x (dim), u (dim)] (AoS, one 16-byte-aligned record per node):
  // the bond pass gathers a neighbour's position and displacement with
  // 16-byte loads.  Double-buffered predicted displacement; x never changes.
  double *xu[2] = {nullptr, nullptr};
  double *v = nullptr, *a = nullptr;
  int cur = 0;                   // xu[cur]: current displacement, xu[cur^1]: predicted next
  int32_t *rp = nullptr;         // canonical CSR, N+1
  int32_t *csr_col = nullptr;    // nnz
  int64_t nnz = 0;
  Sell sell;                     // full lattice, row = node
  double *damage = nullptr;
  int32_t *region_flag = nullptr;  // device flag: a bond in the link region broke
  int32_t *nonfinite_flag = nullptr;  // device, 2 ints (sticky): [0] a non-finite PD velocity at a
                                      // macro-step end, [1] a bounded wait of the subcycle kernel gave up
  hipEvent_t nf_event = nullptr;   // after the copy of nonfinite_flag to pinned_flag[2] (end of mts_advance)
  bool nf_recorded = false;
  uint8_t *in_region = nullptr;    // per node
  int32_t *layer = nullptr;        // per node: smallest h <= m-1 within h horizons of a constraint, else m

  // ---- FE ----
  int nen = 4, ngp = 4, nstr = 3;
  int64_t nfe = 0, ne = 0;
  int32_t *conn = nullptr;       // ne * nen
  uint8_t *eact = nullptr;       // ne
  double *gpa = nullptr;         // ne * ngp
  int32_t *n2e_ptr = nullptr, *n2e = nullptr;  // node -> (element*nen + local) list
  uint8_t *nact = nullptr, *bc = nullptr;
  double *xF = nullptr, *mF = nullptr, *PF = nullptr;
  double *uF = nullptr, *vF = nullptr, *aF = nullptr;
  double *ut = nullptr, *vt = nullptr, *at = nullptr, *fe_buf = nullptr;
  // implicit FE step (fe_beta > 0)
  double fe_beta = 0.0;
  double *fe_Ke = nullptr;        // per element (nen dim)^2 stiffness, alpha-weighted
  uint8_t *fe_free = nullptr;     // per dof: active and not prescribed
  double *fe_inv_diag = nullptr;  // Jacobi preconditioner of M + beta dt^2 K
  double *fe_HF = nullptr;        // nl x nl FE block (dt/2) G_F A^-1 G_F^T of H
  struct FeImplicit *fe_impl = nullptr;  // conjugate-gradient buffers (host struct)
  // implicit PD step (pd_beta > 0, pure-PD mode, FP64)
  double pd_beta = 0.0;
  struct PdImplicit *pd_impl = nullptr;
  void *fe_tab = nullptr;        // element tables (shape functions, derivatives, Hooke), device
  std::vector<int32_t> h_conn;
  std::vector<uint8_t> h_bc;

  // ---- coupling ----
  int64_t nc = 0, nl = 0;
  int32_t *cn = nullptr;         // constraint -> PD node
  int32_t *cidx = nullptr;       // PD node -> constraint or -1
  int32_t *cel = nullptr;        // constraint -> element
  double *cw = nullptr;          // nc * nen interpolation weights N_a(x_p)
  int32_t *f2c_ptr = nullptr, *f2c = nullptr;  // FE node -> (constraint*nen + a)
  int32_t *fe_ring = nullptr;    // FE nodes with constraint entries
  int64_t n_ring = 0;
  double *lam = nullptr, *lam0 = nullptr, *rhs = nullptr;
  double *H = nullptr;           // nl * nl, row-major assembly buffer of H
  // Inverse of H, block-diagonal over connected components of the coupling
  // graph; each block stored as its lower-triangle 64 x 64 tiles.
  struct SymBlocks {
    int64_t n_comp = 0, n_tiles = 0, n_max = 0;
    std::vector<int64_t> h_off;     // component dof offsets (n_comp + 1)
    std::vector<int32_t> h_idx;     // concatenated dof indices
    int32_t *idx = nullptr;         // device copy
    int64_t *off = nullptr;         // device copy of h_off
    int32_t *tile_meta = nullptr;   // per tile: component, I, J
    int64_t *tile_base = nullptr;   // per component: first tile
    double *packed = nullptr;       // n_tiles * 4096
    double *rowpart = nullptr, *colpart = nullptr;  // n_tiles * 64
    double *pv = nullptr, *pw = nullptr;  // sweep panels, 64 x 256 per tile row
    double *pinv = nullptr;         // inverse of the current pivot tile
    double *pblk = nullptr;         // inverse of the current 256-wide pivot block
    int64_t n_rows = 0;             // block rows over all components
    int32_t *row_comp = nullptr, *row_block = nullptr;
    // tiles the multiplier solve reads: every diagonal tile and every tile
    // whose largest entry exceeds kInvDrop of its component's largest entry
    int32_t *kept = nullptr;        // tile ids, ascending
    int64_t n_kept = 0;
    int64_t *n_kept_dev = nullptr;  // the same count on the device (launches read it, so a
                                    // captured solve stays valid when a rebuild changes it)
    double *tile_max = nullptr;     // per tile: largest |entry| of the inverse
    // kept tiles whose largest entry is at most 2^-29 of their component's
    // largest are stored in FP32, in place in the first half of their slot
    uint8_t *kept_f32 = nullptr;    // per kept entry: 1 if stored in FP32
    int64_t n_kept32 = 0;
    bool prune = true;
    // the multiplier solve's right-hand side in component-block order (each
    // component padded with zeros to whole tiles), every dof's position in it,
    // a header per kept tile, and per block row the partial sums of its kept
    // tiles (ascending block column); sized for every tile at setup, so a
    // rebuild rewrites them in place
    double *rperm = nullptr;
    int32_t *rpos = nullptr;
    int4 *hdr = nullptr;        // per kept tile: {tile, rI, rJ, flags (1: FP32, 2: off the diagonal)}
    int32_t *red_off = nullptr; // per block row and reduction wavefront: first entry of red
    int2 *red = nullptr;        // {tile << 1 | (1: column partial), block column}
    std::vector<int64_t> h_pbase;  // per component: first entry in rperm (n_comp + 1)
    int form = 0;                  // solve form: 0 by the kept-tile count, 1 all loads at once, 2 streaming
  } sym;
  std::vector<int32_t> h_cn;
  int64_t n_region = 0;
  Sell rsell;                    // link region rows
  double *Wu[2] = {nullptr, nullptr};
  double *Wxu[2] = {nullptr, nullptr};  // final-update response: node records [x, w], double-buffered
  double *Wv = nullptr, *Wa = nullptr; // dim*N (zero outside the region)
  int64_t n_colors = 0;
  int32_t *ccolor = nullptr;     // colour of each constraint
  int32_t *owner = nullptr;      // n_colors * nc: loaded constraint of that colour reaching q, or -1
  std::vector<int32_t> h_batch_off;  // per batch of unit loads: range of batch_nodes
  int32_t *batch_nodes = nullptr;    // PD node ids of the constraints loaded by each batch
  int32_t *batch_layer = nullptr;    // per link-region slice: layer w.r.t. the current batch's loads
  // further response buffers and streams of a build: its colour batches run
  // on kBuildStreams streams at once (batch b on stream b mod kBuildStreams,
  // with buffer set b mod kBuildStreams; set 0 is Wu, Wv, Wa, batch_layer)
  static constexpr int kBuildStreams = 4;
  struct BuildSet {
    double *u[2] = {nullptr, nullptr}, *v = nullptr, *a = nullptr;
    int32_t *layer = nullptr;
  } bset[kBuildStreams - 1];
  hipStream_t bstream[kBuildStreams - 1] = {};
  hipEvent_t bfork = nullptr, bjoin[kBuildStreams - 1] = {};
  int build_streams = kBuildStreams;
  // rebuilds recompute only the columns whose response support holds a node
  // with a bond changed since the last build (the rest are unchanged bit for bit)
  bool incremental = true;
  uint64_t *built_mask = nullptr;    // full-lattice bond states of the last build
  bool built_valid = false;
  uint8_t *dirty = nullptr;          // per PD node: a bond of its row changed since the last build
  int32_t *ccolor_sub = nullptr;     // colour of each recomputed constraint, -1 for the others
  uint8_t *csel = nullptr;           // per constraint: recomputed by this rebuild
  std::vector<int32_t> h_ccolor;     // host copy of the colours
  std::unordered_map<int64_t, std::vector<int32_t>> h_ccells;  // constraints by cell of size own_r
  double own_r = 0.0;                // reach of a response (with half a horizon of slack)
  int64_t n_rebuild_cols = 0;
  int nrhs = 8;
  bool keep_h = false;
  double *Hcopy = nullptr;       // H before inversion (kept when small, for inspection)
  int32_t *pinned_flag = nullptr;  // host-pinned: [0], [1] rebuild flag per slot, [2], [3] copies of nonfinite_flag
  uint64_t *mask_snap[2] = {nullptr, nullptr};  // full-lattice bond states at the end of a macro step
  hipEvent_t flag_event[2] = {nullptr, nullptr};
  bool pending = false;
  int pending_slot = 0;

  bool verbose = false;
  int force_lanes = 0;             // lanes per row of the full-lattice bond layout (0: pick_lanes)
  int tiled = 1;                   // full layout rows in spatial tile order (shrinks the staged
                                   // neighbour lists of a workgroup)
  int pd_variant = 0;              // bond-pass loop shape (chunk size, pipelining)
  bool halo = true;                // stage neighbour records in LDS when they fit
  int region_lanes = 0;            // lanes per row of the link region layout (0: automatic)
  int subcycle = 0;                // run the m substeps of a macro step as one launch when it fits
                                   // (opt-in: measured slower than one launch per substep)
  uint32_t sub_epoch = 0;          // substeps finished by subcycle launches (workgroup flag numbering)
  uint32_t spin_limit = 1u << 18;  // polls of a subcycle wait before it gives up (tests set it low)
  int sub_capacity = -1;           // co-resident workgroups of the subcycle kernel (-1: not computed)
  int halo_waves = 0;              // wavefronts per workgroup of the staged pass (0: 8 for 3D mixed, else 4)
  double t_create0 = 0.0;

  // profiling
  bool profiling = false;
  bool fe_free_done = false;  // the coming macro step's FE free step is already enqueued
  hipEvent_t ev_start[MTS_KT_COUNT]{}, ev_stop[MTS_KT_COUNT]{};
  struct EvPair {
    hipEvent_t e0, e1;
    int launches;  // back-to-back launches between the two events
  };
  std::vector<EvPair> ev_pending[MTS_KT_COUNT];
  int64_t kt_count[MTS_KT_COUNT]{};
  double kt_ms[MTS_KT_COUNT]{};
  std::vector<hipEvent_t> ev_pool;

  void prof_begin(int k, hipEvent_t *e0);
  void prof_end(int k, hipEvent_t e0, int launches = 1);
  void prof_collect();
};

// neighbour build and bond layout (neighbors.hip)
void build_neighbors(Solver &s);
void build_sell(Solver &s, Sell &out, const std::vector<int32_t> &rows_host, const uint64_t *src_mask_full, int L);
void sell_regather_mask(Solver &s, Sell &out, const uint64_t *src_mask_full);
void sell_coefficients(Solver &s, Sell &out);
void sell_pack_slots(Solver &s, Sell &out, const int32_t *dev_col = nullptr, bool fp64 = false);
void sell_build_halo(Solver &s, Sell &out);
void bonds_to_csr_state(Solver &s, uint8_t *dev_out);
// PD kernels (pd.hip)
void pd_setup(Solver &s);
void pd_predict_all(Solver &s);
void pd_substep(Solver &s, int j);
bool pd_subcycle(Solver &s);  // all m substeps in one launch; false: not applicable, nothing enqueued
void pd_damage(Solver &s);
// batched substeps over several solvers of one form and lane count (pd.hip)
size_t substep_entry_size();
int64_t substep_blocks(const Solver &s);
void substep_entry_fill(Solver &s, int j, int cur, int32_t first_block, void *dst);
void substep_batch_launch(int dim, bool mixed, int L, const void *dev_tab, const int32_t *dev_blk_req,
                          int64_t nblocks, hipStream_t st);
// FE kernels (fe.hip)
void fe_setup(Solver &s);
void fe_free_step(Solver &s);
void fe_correct(Solver &s);
// implicit FE step (fe_implicit.hip)
void fe_implicit_setup(Solver &s);
void fe_implicit_free_step(Solver &s);
void fe_implicit_correct(Solver &s);  // after lambda_m
void fe_implicit_hf(Solver &s);       // the FE block of H, once
void fe_implicit_free(Solver &s);     // host buffers
// implicit PD step (pd_implicit.hip)
void pd_implicit_setup(Solver &s);
void pd_implicit_step(Solver &s);     // one PD step, then the break test on its displacement
void pd_implicit_free(Solver &s);
// coupling (coupling.hip)
void coupling_setup(Solver &s);
void coupling_rebuild(Solver &s, const uint64_t *full_mask);
void coupling_free(Solver &s);  // the build streams and events (memory is the arena's)
// fuse_next_fe: the next macro step's FE free step rides in the link
// launches (its kernels are independent of them); returns whether it did
// snap_slot >= 0: also save this macro step's bond states into that slot and
// clear the rebuild flag (after the caller copied it to the host)
bool coupling_solve_and_correct(Solver &s, bool fuse_next_fe = false, int snap_slot = -1);
void coupling_lambda(Solver &s);  // lambda_m
bool coupling_link(Solver &s, bool fuse_next_fe = false, int snap_slot = -1);  // FE and PD corrections
// independent passes run by extra workgroups of a link launch
enum { kSideNone = 0, kSideRing = 1, kSideElem = 2, kSideGather = 3, kSideSnap = 4 };
// dense linear algebra (dense.hip)
void sym_blocks_setup(Solver &s, const std::vector<std::vector<int32_t>> &comps);
void sym_blocks_build(Solver &s);
// y (and y2) <- H^-1 r, r given in dof order and in component-block order
// (sym.rperm's layout); each form of the solve reads the layout it needs
void sym_blocks_apply(Solver &s, const double *r_dof, const double *r_blk, double *y, double *y2 = nullptr);
void sym_blocks_prune(Solver &s);  // the tiles the solve reads
// solver construction and helpers shared with the serving pool (solver.hip)
void create_impl(const mts_problem *pin, void *stream, Solver *s);
mts_status fail_from_exception();
void set_error(const char *fmt, ...);
void check_finite(Solver &s);
void resolve_pending(Solver &s);
void snapshot_states(Solver &s, int slot);
void snapshot_masks(Solver &s, int slot);  // the bond states and the flag clear only
mts_status read_impl(Solver &s, int32_t what, double *out, int64_t cap, int64_t *n);
mts_status read_device_impl(Solver &s, int32_t what, double *dev_out, int64_t cap, int64_t *n);
// energies and broken-bond count of the current state (energy.hip)
int64_t count_intact(Solver &s);
void energy_impl(Solver &s, mts_energy_info *out);
void energy_noalloc_impl(Solver &s, double *dev_out);  // partial sums in a static device buffer
void query_impl(Solver &s, mts_info *o);
// progress log on stderr when MTS_VERBOSE is set
void vlog(const Solver &s, const char *fmt, ...);
// scans (neighbors.hip)
void exclusive_scan_i64(hipStream_t st, DeviceArena &ar, const int64_t *in, int64_t *out, int64_t n);

}  // namespace mts
