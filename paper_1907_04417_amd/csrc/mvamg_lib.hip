// C ABI of the MI355X solve phase (declared in include/mvamg.h): hierarchy
// upload, V-cycle (Section 5: forward/backward Gauss-Seidel, block-diagonal
// multiple-vector transfers of Section 4, exact coarsest solve) and
// preconditioned CG with the paper's stopping rule (Section 5).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "hier_host.hpp"
#include "dense.hpp"
#include "kernels.hpp"
#include "kernels_multi.hpp"
#include "setup_kernels.hpp"
#include "mini_kernels.hpp"
#include "mvamg.h"

using namespace mvamg;

struct mvamg_hier_host {
  HostHier h;
};

namespace {

thread_local std::string g_err;

void hipcheck(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(MVAMG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHECK(x) hipcheck((x), #x)
#define LAUNCHCHECK(name) hipcheck(hipGetLastError(), name)

// grid of a grid-stride kernel whose block partials are reduced afterwards
int grid_for(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  return (int)b;
}

// grid of a pure elementwise kernel: one element per thread
int grid_elem(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return (int)b;
}

struct DevLevel {
  int n = 0;
  bool sell = false;
  int G = 8;   // kernel instantiation of a grouped level: 64 / G lanes per row (autotuned, >= G0)
  int G0 = 8;  // smallest admissible G: the level's largest group rounded up to a power of two
  bool wide = false;  // grouped level: one block of kWide threads per group (autotuned)
  bool gshared = false;  // grouped level whose groups all share one column list per group
  int ng = 0, ns = 0, nslabs = 0;
  int rows0 = 0;  // rows of stage 0 (point levels)
  std::vector<int> h_sgrp, h_sslab;
  std::vector<int> h_srow;  // first row of every stage (nstages + 1 entries)
  int64_t nent = 0;    // stored off-group entries (with padding)
  int64_t nnz = 0;     // stored entries of A_l (file), for byte counts
  std::vector<int64_t> stage_rows, stage_nnz;
  int64_t ndblk = 0;
  // device arrays
  Slab* slabs = nullptr;
  // sliced ELL: the slabs again, in the order of the file index of their
  // first row (for a grid numbering, spatial order), for the block kernels
  // that sweep many stages at once: all stages (bslab_full) or all but the
  // last (bslab_part, nslab_part of them).  Neighbouring rows of different
  // colours are then handled close in time, by the same XCD.
  Slab *bslab_full = nullptr, *bslab_part = nullptr;
  int nslab_part = 0;
  int* rowptr = nullptr;
  int* rec = nullptr;  // per group: 16-int record (first row, rows, block offset, row entry offsets)
  int* col = nullptr;
  uint16_t* col16 = nullptr;  // sliced ELL: 16-bit column deltas, lane-packed (see SellCols)
  int* pk = nullptr;          // sliced ELL: per slab, offset of its lane-packed deltas and codes
  int* cbase = nullptr;
  int* scb = nullptr;
  int64_t nnz16 = 0;                 // stored entries in 16-bit slabs
  std::vector<int64_t> stage_nnz16;  // the same per stage
  std::vector<int64_t> stage_later;  // grouped levels: entries of a stage's rows in later stages
  // grouped levels: per stage, the stored column indices (shared group
  // lists) and those of later-stage columns
  std::vector<int64_t> stage_gidx, stage_later_idx;
  int64_t gidx = 0;
  int* gcol = nullptr;  // grouped levels: the column index lists the single-vector kernels read
  // sliced-ELL levels with few distinct values: 1-byte codes of the entries
  // and of the diagonal, and their tables (binary64 and binary32); valid
  // for the values uploaded with the layout, cleared by a value refill
  uint8_t *vcode = nullptr, *dcode = nullptr;
  double *vtab = nullptr, *dtab = nullptr;
  float *vtab32 = nullptr, *dtab32 = nullptr;
  int nvtab = 0, ndtab = 0;
  bool vcoded = false, dcoded = false;
  double* val = nullptr;
  float* val32 = nullptr;
  int* src = nullptr;
  int* gstart = nullptr;
  int* dboff = nullptr;
  double* dblk = nullptr;
  float* dblk32 = nullptr;
  int* dsrc = nullptr;
  double* diag = nullptr;  // point levels: the diagonal (alias of dblk)
  float* diag32 = nullptr;
  double* dl1 = nullptr;
  float* dl1_32 = nullptr;
  // work vectors
  double *r = nullptr, *x = nullptr, *s = nullptr;
  float *r32 = nullptr, *x32 = nullptr, *s32 = nullptr;
  // batch, level 0: problem of every slab and of every row (smoother order)
  int* slabprob = nullptr;
  int* rowprob = nullptr;
  // K-cycle, levels 1 .. nl - 2 (binary64): the inner iterations' vectors
  // (A c1, the second residual, the second direction c2 and A c2; c1 is x)
  // and their five scalars
  double *kv1 = nullptr, *kr2 = nullptr, *kc2 = nullptr, *kv2 = nullptr, *ks = nullptr;
  // block work vectors (n x 32, allocated on the first block call)
  double *br = nullptr, *bx = nullptr, *bs = nullptr;
  float *br32 = nullptr, *bx32 = nullptr, *bs32 = nullptr;
};

struct DevTransfer {
  int nagg = 0;
  int* arows = nullptr;  // member rows of every aggregate (level order), runs given by the records
  int* arec = nullptr;  // per-aggregate records (kARec ints each)
  int* aprob = nullptr; // batch, level 0: problem of every aggregate
  int nf = 0, kmax = 1;  // fine rows, widest block
  // Point fine level: a Gauss-Seidel row update does not read the row's own
  // value, so the rows [ncut, nf) of the last stage -- the first one the
  // backward sweep after the prolongation relaxes -- are overwritten before
  // anything reads them, and the prolongation stops at ncut (nu_cut U entries
  // lie in the rows before it).  ncut = nf on levels with multi-row groups.
  int ncut = 0;
  int64_t nu_cut = 0;
  // U entries of the rows before the first row of the level's last stage
  // (the rows a restriction after a Gauss-Seidel sweep reads on a point level)
  int64_t nu_scut = 0;
  int64_t nu = 0;        // entries of the U blocks
  int* cinfo = nullptr;  // per fine row: 8 * first coarse row + (k - 1)
  double* Urow = nullptr;  // per fine row, column-major [q * nf + row]
  float* Urow32 = nullptr;
  double* U = nullptr;
  float* U32 = nullptr;
};

struct DevCoarse {
  int n = 0, np = 0;         // size, padded size (multiple of 64) of a single block
  int nb = 1;                // diagonal blocks (one per problem of a batch)
  double* Ainv = nullptr;    // np x np row-major inverse; a batch: the blocks' inverses one after another
  int *cprob = nullptr, *coff = nullptr, *cnp = nullptr;  // batch: row -> block, block rows, padded sizes
  int64_t* aoff = nullptr;   // batch: offset of each block's inverse
  double ainv_entries = 0.0; // sum of the blocks' n_b^2 (algorithmic bytes / 8)
  double *r = nullptr, *z = nullptr;
  double *br = nullptr, *bz = nullptr;  // block vectors for the binary32 block cycle
  double* bsplit = nullptr;             // partial products of a split block product
  // single problem: the inverse's lower-triangle 64 x 64 tiles for the
  // symmetric product (half the bytes of Ainv), their (I, J), the slots of
  // the first pass
  int nt = 0, ntiles = 0;
  double* tiles = nullptr;
  int2* tij = nullptr;
  double* spart = nullptr;
};

// per-system scalars and partials of the multi-system solves
struct MultiBufs {
  int nsys = 0, nparts = 0;
  double* scal = nullptr;    // nsys * S_NSCAL
  double* part = nullptr;    // 2 * nsys * nparts
  double* act = nullptr;     // nsys flags staged for k_mset_active
  double* pinned = nullptr;  // host copy of scal
  double* pact = nullptr;    // host staging of act
};

}  // namespace

struct mvamg_hier {
  int device = 0;
  int nl = 0, n = 0;
  int64_t nnz = 0;
  std::vector<int> lev_n;
  std::vector<int64_t> lev_nnz;
  std::vector<DevLevel> lv;  // nl entries; the last holds only work vectors
  std::vector<DevTransfer> tr;
  DevCoarse co;
  int* perm0 = nullptr;  // level-0 new -> file index
  int* frp = nullptr;    // file CSR pattern of level 0
  int* fci = nullptr;
  double* fval = nullptr;  // the level-0 values in use, file CSR order
  int* cmpflag = nullptr;  // two flags of the matrix check (pattern, values)
  // CG vectors (binary64, level-0 smoother order)
  double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double* scal = nullptr;
  double* part = nullptr;
  int dot_nparts = 0;  // partials of z.r written by the last cycle's fine backward sweep
  double* pinned = nullptr;  // host copies of scal, two slots (mapped; see cg_step_a)
  double* pinned_dev = nullptr;
  // batch of independent problems (nprob > 0): level-0 rows of problem p are
  // the file rows [poff[p], poff[p+1]); iperm0 maps a file row to smoother order
  int nprob = 0;
  int pchunks = 1;
  std::vector<int> h_poff;
  // batch with problems on the one-launch small-problem path: the caller's
  // view (all problems, their row offsets), which of them form the lockstep
  // part above (uid) and which the small path (mid), and the small path's data
  int nall = 0;
  std::vector<int> h_aoff, uid, mid;
  int* umap = nullptr;  // lockstep part's row -> caller's row
  int nmini = 0, mini_maxit = 0;
  MiniProb* mprobs = nullptr;
  MiniLevel* mlevs = nullptr;
  int* mints = nullptr;
  double *mdbls = nullptr, *mwork = nullptr, *mhist = nullptr;
  MiniInfo* minfo = nullptr;
  hipStream_t mstream = nullptr;
  hipEvent_t mev[2] = {nullptr, nullptr};
  int* poff = nullptr;
  int* iperm0 = nullptr;
  // while set (batch CG iterations), level-0 kernels skip the work units of
  // problems whose S_ACT flag (at skip_act + S_NSCAL * problem) is zero
  const double* skip_act = nullptr;
  double skip_frac = 1.0;  // meanwhile: fraction of level-0 rows still worked on (byte accounting)
  // several systems at once
  MultiBufs mb;
  bool blk_ready = false;
  int gemm_variant = -1;  // coarsest block product variant (-1: default; autotuned)
  double *bb = nullptr, *bxv = nullptr, *bp = nullptr, *bq = nullptr;  // level-0 block CG vectors
  hipStream_t cap = nullptr;              // stream used only to capture graphs
  std::map<int, hipGraphExec_t> graphs;   // one CG iteration per (precision, smoother)
  bool use_graphs = true;
  hipEvent_t itev[2] = {nullptr, nullptr};  // ends of the CG steps in flight (one ahead of the host)
  // measurement: per-launch HIP events for every instrumented kernel
  bool prof = false;
  // byte booking while measuring: false, the compact forms the kernels read
  // (value codes, 2-byte column deltas, shared group lists); true, the plain
  // model (every stored entry a value and a 4-byte index, the coarsest
  // inverse whole)
  bool book_plain = false;
  std::vector<hipEvent_t> ev_pool;
  struct Pending {
    int kc;
    hipEvent_t e0, e1;
    double bytes;
  };
  std::vector<Pending> pending;
  int64_t kc_launches[MVAMG_KC_COUNT] = {};
  double kc_ms[MVAMG_KC_COUNT] = {}, kc_bytes[MVAMG_KC_COUNT] = {};
  // Device memory: every array lives in the caller's arena (mvamg_upload).
  // Allocation bumps an offset; a release of the newest live arrays gives
  // their space back (the coarsest factorisation's temporaries).  With no
  // arena base the handle only sizes: nothing touches the device, and
  // arena_peak ends as the bytes an arena needs.
  unsigned char* arena = nullptr;
  size_t arena_cap = 0, arena_top = 0, arena_peak = 0;
  struct Live {
    size_t off, end;
    bool freed;
  };
  std::vector<Live> live;
  bool sizing() const { return arena == nullptr; }
  // while sizing, addresses start at a non-null value that nothing dereferences
  uintptr_t arena_base() const { return sizing() ? (uintptr_t)4096 : reinterpret_cast<uintptr_t>(arena); }

  template <typename T>
  T* dalloc(size_t count) {
    if (count == 0) count = 1;
    const size_t off = (arena_top + 255) / 256 * 256, end = off + count * sizeof(T);
    if (!sizing() && end > arena_cap)
      throw Error(MVAMG_ERR_ARG, "device arena of " + std::to_string(arena_cap) +
                                     " bytes is too small for this handle (size it with mvamg_arena_bytes)");
    arena_top = end;
    arena_peak = std::max(arena_peak, end);
    live.push_back({off, end, false});
    // while sizing, a distinct non-null address that nothing dereferences
    return reinterpret_cast<T*>(arena_base() + off);
  }
  void dfree(void* ptr) {
    const size_t off = (size_t)(reinterpret_cast<uintptr_t>(ptr) - arena_base());
    for (auto& a : live)
      if (a.off == off && !a.freed) a.freed = true;
    while (!live.empty() && live.back().freed) live.pop_back();
    arena_top = live.empty() ? 0 : live.back().end;
  }
  // whether arrays of these byte counts, taken in order, fit the arena
  bool fits(const std::vector<size_t>& bytes) const {
    if (sizing()) return true;
    size_t top = arena_top;
    for (size_t b : bytes) top = (top + 255) / 256 * 256 + std::max<size_t>(b, 1);
    return top <= arena_cap;
  }
  template <typename T>
  T* upload_vec(const std::vector<T>& v, hipStream_t st) {
    T* d = dalloc<T>(v.size());
    if (!v.empty() && !sizing())
      HIPCHECK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return d;
  }
  ~mvamg_hier() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (auto& pd : pending) {
      (void)hipEventDestroy(pd.e0);
      (void)hipEventDestroy(pd.e1);
    }
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    if (cap) (void)hipStreamDestroy(cap);
    if (mstream) (void)hipStreamDestroy(mstream);
    for (hipEvent_t e : mev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : itev)
      if (e) (void)hipEventDestroy(e);
    if (pinned) (void)hipHostFree(pinned);
    if (mb.pinned) (void)hipHostFree(mb.pinned);
    if (mb.pact) (void)hipHostFree(mb.pact);
  }
};

namespace {

Red mkred(mvamg_hier* h) { return Red{h->part}; }

enum SkipUnit { SKIP_SLAB, SKIP_ROW, SKIP_AGG };

// algorithmic bytes of a level-l launch that skips stopped problems
double skip_bytes(const mvamg_hier* h, int l, double bytes) { return (l == 0 && h->skip_act) ? bytes * h->skip_frac : bytes; }

Skip lskip(const mvamg_hier* h, int l, SkipUnit u) {
  if (l != 0 || !h->skip_act) return Skip{nullptr, nullptr};
  const int* up = (u == SKIP_SLAB) ? h->lv[0].slabprob : (u == SKIP_ROW) ? h->lv[0].rowprob : h->tr[0].aprob;
  if (!up) return Skip{nullptr, nullptr};
  return Skip{up, h->skip_act};
}

hipEvent_t take_event(mvamg_hier* h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHECK(hipEventCreate(&e));
  return e;
}

// Launches kern; while measurement is on, the launch carries start/stop
// events (AMD's extended launch) and its algorithmic bytes are booked to
// kernel class kc.
template <typename... KArgs, typename... Args>
void klaunch(mvamg_hier* h, int kc, double bytes, void (*kern)(KArgs...), dim3 grid, dim3 block, hipStream_t st,
             Args... args) {
  static_assert(sizeof...(KArgs) == sizeof...(Args), "argument count");
  if (h->prof) {
    hipEvent_t e0 = take_event(h), e1 = take_event(h);
    hipExtLaunchKernelGGL(kern, grid, block, 0, st, e0, e1, 0, static_cast<KArgs>(args)...);
    h->pending.push_back({kc, e0, e1, bytes});
  } else {
    hipLaunchKernelGGL(kern, grid, block, 0, st, static_cast<KArgs>(args)...);
  }
}

// Books the finished measured launches (the stream has been synchronised).
void harvest(mvamg_hier* h) {
  for (auto& pd : h->pending) {
    float ms = 0.0f;
    HIPCHECK(hipEventElapsedTime(&ms, pd.e0, pd.e1));
    h->kc_launches[pd.kc] += 1;
    h->kc_ms[pd.kc] += ms;
    h->kc_bytes[pd.kc] += pd.bytes;
    h->ev_pool.push_back(pd.e0);
    h->ev_pool.push_back(pd.e1);
  }
  h->pending.clear();
}

// Adds the block partials of the previous kernel (grid blocks) and applies
// `mode`; host: also copies the scalars there (mapped host memory).
void finish(mvamg_hier* h, int nv, int grid, int mode, hipStream_t st, double* host = nullptr) {
  if (nv == 1)
    k_finish<1><<<1, kFinish, 0, st>>>(grid, h->part, h->scal, mode, host);
  else
    k_finish<2><<<1, kFinish, 0, st>>>(grid, h->part, h->scal, mode, host);
  LAUNCHCHECK("finish");
}

// --------------------------------------------------------- level operators

template <typename T>
const T* lval(const DevLevel& L);
template <>
const double* lval<double>(const DevLevel& L) {
  return L.val;
}
template <>
const float* lval<float>(const DevLevel& L) {
  return L.val32;
}
template <typename T>
const T* ldblk(const DevLevel& L);
template <>
const double* ldblk<double>(const DevLevel& L) {
  return L.dblk;
}
template <>
const float* ldblk<float>(const DevLevel& L) {
  return L.dblk32;
}
template <typename T>
SellVals<T> svals(const DevLevel& L) {
  SellVals<T> V{lval<T>(L), ldblk<T>(L), L.vcoded ? L.vcode : nullptr, L.dcoded ? L.dcode : nullptr, nullptr, nullptr,
                L.nvtab, L.ndtab};
  if constexpr (std::is_same<T, double>::value) {
    V.vtab = L.vtab;
    V.dtab = L.dtab;
  } else {
    V.vtab = L.vtab32;
    V.dtab = L.dtab32;
  }
  return V;
}

// Bytes of the matrix data the single-vector kernels read for rows rows with
// nnz entries (nnz16 of them off-diagonal with 2-byte indices) of a
// sliced-ELL level: values or codes, indices, diagonal.
template <typename T>
double sell_mat_bytes(const mvamg_hier* h, const DevLevel& L, double nnz, double rows, double nnz16) {
  if (h->book_plain) return nnz * (sizeof(T) + 4.0);
  const double vb = L.vcoded ? 1.0 : sizeof(T), db = L.dcoded ? 1.0 : sizeof(T);
  return (nnz - rows) * (vb + 4.0) - 2.0 * nnz16 + rows * db;
}

template <typename T>
const T* ldl1(const DevLevel& L);
template <>
const double* ldl1<double>(const DevLevel& L) {
  return L.dl1;
}
template <>
const float* ldl1<float>(const DevLevel& L) {
  return L.dl1_32;
}
template <typename T>
const T* tUrow(const DevTransfer& P);
template <>
const double* tUrow<double>(const DevTransfer& P) {
  return P.Urow;
}
template <>
const float* tUrow<float>(const DevTransfer& P) {
  return P.Urow32;
}
template <typename T>
const T* tU(const DevTransfer& P);
template <>
const double* tU<double>(const DevTransfer& P) {
  return P.U;
}
template <>
const float* tU<float>(const DevTransfer& P) {
  return P.U32;
}
template <typename T>
T* lr(DevLevel& L);
template <>
double* lr<double>(DevLevel& L) {
  return L.r;
}
template <>
float* lr<float>(DevLevel& L) {
  return L.r32;
}
template <typename T>
T* lx(DevLevel& L);
template <>
double* lx<double>(DevLevel& L) {
  return L.x;
}
template <>
float* lx<float>(DevLevel& L) {
  return L.x32;
}
template <typename T>
T* ls(DevLevel& L);
template <>
double* ls<double>(DevLevel& L) {
  return L.s;
}
template <>
float* ls<float>(DevLevel& L) {
  return L.s32;
}

// algorithmic bytes of one smoother stage: every stored entry of its rows
// (value + 4-byte index, 2-byte in 16-bit slabs), and per row an index, r,
// x written and x read
// Column index bytes the single-vector kernels read for stage c: 4 or 2
// (16-bit slabs) per entry on point levels, 4 per stored list entry on
// grouped levels.
double stage_idx_bytes(const mvamg_hier* h, const DevLevel& L, int c) {
  if (h->book_plain) return 4.0 * L.stage_nnz[c];
  return L.sell ? 4.0 * L.stage_nnz[c] - 2.0 * L.stage_nnz16[c] : 4.0 * L.stage_gidx[c];
}

template <typename T>
double stage_bytes(const mvamg_hier* h, const DevLevel& L, int c) {
  if (L.sell)
    return sell_mat_bytes<T>(h, L, L.stage_nnz[c], L.stage_rows[c], L.stage_nnz16[c]) +
           (double)L.stage_rows[c] * (4 + 2 * sizeof(T));
  return (double)L.stage_nnz[c] * sizeof(T) + stage_idx_bytes(h, L, c) + (double)L.stage_rows[c] * (4 + 3 * sizeof(T));
}

SellCols scols(const DevLevel& L) { return SellCols{L.col, L.col16, L.cbase, L.scb, L.pk}; }

// first_sweep: forward sweep from x = 0 (entries of later stages skipped;
// see k_gs_sell and k_gs_grp).  dot_part (binary64 sliced-ELL levels): the
// stage also writes block partials of x.r for its rows there.  Returns the
// number of partials written.
template <typename T>
int gs_stage(mvamg_hier* h, int l, const DevLevel& L, int c, const T* r, T* x, int backward, hipStream_t st,
             bool first_sweep = false, double* dot_part = nullptr) {
  const int kc = (l == 0) ? MVAMG_KC_SMOOTH_FINE : MVAMG_KC_SMOOTH_COARSE;
  const bool gfirst = first_sweep && !L.sell && !backward;
  // entries of later stages, not read by a grouped level's forward sweep from
  // zero (stage_later and stage_later_idx exist on grouped levels only)
  const double later = gfirst ? (double)L.stage_later[c] * sizeof(T) +
                                    4.0 * (h->book_plain ? (double)L.stage_later[c] : (double)L.stage_later_idx[c])
                              : 0.0;
  const double by = skip_bytes(h, l, stage_bytes<T>(h, L, c) - later);
  if (L.sell) {
    const int s0 = L.h_sslab[c], s1 = L.h_sslab[c + 1];
    if (s1 <= s0) return 0;
    const int grid = (s1 - s0 + 3) / 4;
    const int lim = first_sweep ? L.h_srow[c] : INT_MAX;
    if constexpr (std::is_same<T, double>::value) {
      if (dot_part) {
        klaunch(h, kc, by, k_gs_sell<T, 1>, grid, kBlock, st, L.slabs, s0, s1, scols(L), svals<T>(L), r, x,
                lskip(h, l, SKIP_SLAB), lim, dot_part);
        LAUNCHCHECK("gs_stage");
        return grid;
      }
    }
    klaunch(h, kc, by, k_gs_sell<T, 0>, grid, kBlock, st, L.slabs, s0, s1, scols(L), svals<T>(L), r, x,
            lskip(h, l, SKIP_SLAB), lim, (double*)nullptr);
  } else {
    const int g0 = L.h_sgrp[c], g1 = L.h_sgrp[c + 1];
    if (g1 <= g0) return 0;
    const int grid = L.wide ? g1 - g0 : (g1 - g0 + 3) / 4;
#define MVAMG_GS_GRP(K)                                                                                                 \
  if (L.wide)                                                                                                           \
    (backward ? klaunch(h, kc, by, k_gs_grp_wide<T, K, 1>, grid, kWide, st, g0, g1, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, 0) \
              : klaunch(h, kc, by, k_gs_grp_wide<T, K, 0>, grid, kWide, st, g0, g1, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, (int)gfirst)); \
  else                                                                                                                  \
    (backward ? klaunch(h, kc, by, k_gs_grp<T, K, 1>, grid, kBlock, st, g0, g1, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, 0) \
              : klaunch(h, kc, by, k_gs_grp<T, K, 0>, grid, kBlock, st, g0, g1, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, (int)gfirst))
    switch (L.G) {
      case 1: MVAMG_GS_GRP(1); break;
      case 2: MVAMG_GS_GRP(2); break;
      case 4: MVAMG_GS_GRP(4); break;
      default: MVAMG_GS_GRP(8); break;
    }
#undef MVAMG_GS_GRP
  }
  LAUNCHCHECK("gs_stage");
  return 0;
}

// First step of the forward sweep from x = 0.  Point levels: x = r / d on
// stage 0 only (later stages skip the unset rows); grouped levels: stage-0
// groups solve their lower-triangular block and every other row is zeroed.
template <typename T>
void zero_stage0(mvamg_hier* h, int l, const DevLevel& L, const T* r, T* x, hipStream_t st) {
  const int kc = (l == 0) ? MVAMG_KC_SMOOTH_FINE : MVAMG_KC_SMOOTH_COARSE;
  if (L.sell) {
    const double by = skip_bytes(h, l, (double)L.rows0 * (2 * sizeof(T) + (L.dcoded && !h->book_plain ? 1 : sizeof(T))));
    klaunch(h, kc, by, k_stage0_point<T>, grid_elem(L.rows0), kBlock, st, L.rows0, svals<T>(L), r, x,
            lskip(h, l, SKIP_ROW));
  } else {
    const double by = skip_bytes(h, l, (double)L.n * sizeof(T) + (double)L.stage_rows[0] * (2 * sizeof(T)));
    klaunch(h, kc, by, k_zero_stage0_grp<T>, grid_for(L.ng), kBlock, st, L.ng, L.h_sgrp[1], L.gstart, L.dboff, ldblk<T>(L), r, x);
  }
  LAUNCHCHECK("zero_stage0");
}

int resid_grid(const DevLevel& L);

// Bytes of the residual over the rows of stages [0, nst); compact: the
// kernels read the compact index forms (16-bit slab entries, shared group
// lists), not 4 bytes per entry.
template <typename T>
double resid_stage_bytes(const mvamg_hier* h, const DevLevel& L, int nst, double vec_bytes, bool compact) {
  compact = compact && !h->book_plain;
  double b = 0.0;
  for (int c = 0; c < nst; ++c)
    b += (compact && L.sell)
             ? sell_mat_bytes<T>(h, L, L.stage_nnz[c], L.stage_rows[c], L.stage_nnz16[c]) +
                   (double)L.stage_rows[c] * (4 + vec_bytes)
             : (double)L.stage_nnz[c] * sizeof(T) + (compact ? stage_idx_bytes(h, L, c) : 4.0 * L.stage_nnz[c]) +
                   (double)L.stage_rows[c] * (4 + vec_bytes);
  return b;
}

// MODE 0: s = r - A x;  MODE 1: s = A x and x.s reduced into scal by `mode`;  MODE 2: s = A x.
// nst >= 0 (MODE 0): only the rows of stages [0, nst) (the rest of s is not
// written).
template <typename T, int MODE>
void resid(mvamg_hier* h, int l, const DevLevel& L, const T* r, const T* x, T* s, int mode, hipStream_t st,
           int nst = -1) {
  const Red red = mkred(h);
  // the CG product is the finest level's; products inside a cycle are residual work
  const int kc = (MODE != 0 && l == 0) ? MVAMG_KC_SPMV : MVAMG_KC_RESIDUAL;
  const bool part = MODE == 0 && nst >= 0 && nst < L.ns;
  const double by = skip_bytes(h, l, part ? resid_stage_bytes<T>(h, L, nst, 3.0 * sizeof(T), true)
                                          : (L.sell ? sell_mat_bytes<T>(h, L, L.nnz, L.n, L.nnz16)
                                                    : (double)L.nnz * sizeof(T) +
                                                          4.0 * (h->book_plain ? (double)L.nnz : (double)L.gidx)) +
                                                4.0 * (L.n + 1) +
                                                (double)L.n * sizeof(T) * (MODE != 0 ? 2 : 3));
  if (L.sell) {
    const int ns = part ? L.h_sslab[nst] : L.nslabs;
    if (ns > 0)
      klaunch(h, kc, by, k_resid_sell<T, MODE>, (ns + 3) / 4, kBlock, st, L.slabs, ns, scols(L), svals<T>(L), r, x,
              s, red, lskip(h, l, SKIP_SLAB));
  } else {
    const int ng = part ? L.h_sgrp[nst] : L.ng;
    const int grid = (ng + 3) / 4;
    if (MODE == 0 && L.wide && ng > 0) switch (L.G) {
      case 1: klaunch(h, kc, by, k_resid_grp_wide<T, 1>, ng, kWideResid, st, ng, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, s); break;
      case 2: klaunch(h, kc, by, k_resid_grp_wide<T, 2>, ng, kWideResid, st, ng, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, s); break;
      case 4: klaunch(h, kc, by, k_resid_grp_wide<T, 4>, ng, kWideResid, st, ng, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, s); break;
      default: klaunch(h, kc, by, k_resid_grp_wide<T, 8>, ng, kWideResid, st, ng, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, s); break;
    }
    else if (ng > 0) switch (L.G) {
      case 1: klaunch(h, kc, by, k_resid_grp<T, 1, MODE>, grid, kBlock, st, ng, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, s, red); break;
      case 2: klaunch(h, kc, by, k_resid_grp<T, 2, MODE>, grid, kBlock, st, ng, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, s, red); break;
      case 4: klaunch(h, kc, by, k_resid_grp<T, 4, MODE>, grid, kBlock, st, ng, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, s, red); break;
      default: klaunch(h, kc, by, k_resid_grp<T, 8, MODE>, grid, kBlock, st, ng, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, s, red); break;
    }
  }
  LAUNCHCHECK("resid");
  if (MODE == 1) finish(h, 1, resid_grid(L), mode, st);
}

int resid_grid(const DevLevel& L) {
  if (L.sell) return (L.nslabs + 3) / 4;
  return (L.ng + 3) / 4;
}

template <typename T>
void coarse_solve(mvamg_hier* h, const T* r, T* z, hipStream_t st);

template <>
void coarse_solve<double>(mvamg_hier* h, const double* r, double* z, hipStream_t st) {
  // z = A_L^{-1} r with the inverse formed at upload from the Cholesky factor
  DevCoarse& C = h->co;
  if (C.nb == 1) {
    // algorithmic bytes: the inverse's lower triangle and the two vectors,
    // booked to the tile pass; the slot sums are overhead of the split
    klaunch(h, MVAMG_KC_COARSE, (h->book_plain ? 8.0 * C.n * (double)C.n : 4.0 * C.n * (C.n + 1.0)) + 16.0 * C.n,
            k_symv_tiles, C.ntiles, kBlock, st, C.n,
            C.nt, (const int2*)C.tij, (const double*)C.tiles, r, C.spart);
    klaunch(h, MVAMG_KC_COARSE, 0.0, k_symv_sum, C.nt, kBlock, st, C.n, C.nt, (const double*)C.spart, z);
  } else
    klaunch(h, MVAMG_KC_COARSE, 8.0 * C.ainv_entries + 16.0 * C.n, k_gemv_batch, (C.n + 3) / 4, kBlock, st, C.n,
            C.cprob, C.coff, C.cnp, C.aoff, C.Ainv, r, z);
  LAUNCHCHECK("coarse_solve");
}

template <>
void coarse_solve<float>(mvamg_hier* h, const float* r, float* z, hipStream_t st) {
  DevCoarse& C = h->co;
  k_cast<float, double><<<grid_for(C.n), kBlock, 0, st>>>(C.n, r, C.r);
  coarse_solve<double>(h, C.r, C.z, st);
  k_cast<double, float><<<grid_for(C.n), kBlock, 0, st>>>(C.n, C.z, z);
  LAUNCHCHECK("coarse_solve32");
}

// x = B_l r (one V-cycle from a zero guess).  x_started: the restriction of
// the finer level has already performed the first pre-smoothing step on x.
// stage0_written (point level): the first stage of the sweep from zero is
// already in x (written with r by the CG update), the other rows are not set.
// dot_part: the backward sweep of this level also writes the block partials
// of x.r (binary64 sliced-ELL level, Gauss-Seidel); their count goes to
// h->dot_nparts.
template <typename T>
void kc_fcg2(mvamg_hier* h, int m, const T* g, T* y, int smoother, hipStream_t st, bool y_started);

// kcyc: the K-cycle -- the coarse correction on a level that is not the
// coarsest is two flexible-CG iterations preconditioned by the K-cycle of
// that level (kc_fcg2), not one recursive cycle.
template <typename T>
void vcycle(mvamg_hier* h, int l, const T* r, T* x, int smoother, hipStream_t st, bool x_started = false,
            double* dot_part = nullptr, bool stage0_written = false, bool kcyc = false) {
  if (l == h->nl - 1) {
    coarse_solve<T>(h, r, x, st);
    return;
  }
  DevLevel& L = h->lv[l];
  DevLevel& C = h->lv[l + 1];
  const DevTransfer& P = h->tr[l];
  T* s = ls<T>(L);
  T* rc = lr<T>(C);
  T* xc = lx<T>(C);
  // pre-smoothing: one forward sweep from x = 0
  if (smoother == MVAMG_SMOOTH_GS) {
    if (!x_started && !stage0_written) zero_stage0<T>(h, l, L, r, x, st);
    // from zero: a point level's forward stages skip later-stage columns when
    // its stage 0 was just written by zero_stage0, a grouped level's always
    // (its other groups are zero either way)
    for (int c = 1; c < L.ns; ++c) gs_stage<T>(h, l, L, c, r, x, 0, st, L.sell ? !x_started : true);
  } else if (!x_started) {
    k_l1_init<T><<<grid_for(L.n), kBlock, 0, st>>>(L.n, ldl1<T>(L), r, x);
  }
  // residual, restriction (fused with the first smoothing step of the next
  // level).  After a Gauss-Seidel sweep, a row of a point level's last stage
  // has zero residual: its neighbours all lie in earlier stages and have not
  // changed since its update.  Those rows are neither computed nor restricted.
  const bool zero_last = smoother == MVAMG_SMOOTH_GS && L.ng == L.n;
  resid<T, 0>(h, l, L, r, x, s, M_NONE, st, zero_last ? L.ns - 1 : -1);
  const int scut = zero_last ? L.h_srow[L.ns - 1] : L.n;
  // 16 lanes per aggregate when there are enough aggregates to fill the GPU,
  // else a wave each
  const bool narrow = P.nagg >= 8192;
  const int tg = narrow ? (P.nagg + 15) / 16 : (P.nagg + 3) / 4;
  const double tby = skip_bytes(h, l, (double)(scut == L.n ? P.nu : P.nu_scut) * sizeof(T) + 4.0 * L.n +
                                          (double)scut * sizeof(T) + (double)C.n * sizeof(T));
  const bool next_smoothed = (l + 2 < h->nl);
  const int init = !next_smoothed ? 0 : (smoother == MVAMG_SMOOTH_GS ? 1 : 2);
  const double iby = next_smoothed ? skip_bytes(h, l, (double)C.n * sizeof(T)) : 0.0;
  const T* cdblk = init == 1 ? ldblk<T>(C) : nullptr;
  const T* cdl1 = init == 2 ? ldl1<T>(C) : nullptr;
  T* xcs = init != 0 ? xc : nullptr;
  const Skip ask = lskip(h, l, SKIP_AGG);
#define MVAMG_RESTRICT_L(KM, LPA)                                                                                 \
  switch (init) {                                                                                                 \
    case 0: klaunch(h, MVAMG_KC_RESTRICT, tby, k_restrict<T, KM, 0, LPA>, tg, kBlock, st, P.nagg, P.arec,       \
                    P.arows, tU<T>(P), s, scut, rc, cdblk, cdl1, xcs, ask); break;                               \
    case 1: klaunch(h, MVAMG_KC_RESTRICT, tby + iby, k_restrict<T, KM, 1, LPA>, tg, kBlock, st, P.nagg, P.arec, \
                    P.arows, tU<T>(P), s, scut, rc, cdblk, cdl1, xcs, ask); break;                               \
    default: klaunch(h, MVAMG_KC_RESTRICT, tby + iby, k_restrict<T, KM, 2, LPA>, tg, kBlock, st, P.nagg,        \
                     P.arec, P.arows, tU<T>(P), s, scut, rc, cdblk, cdl1, xcs, ask); break;                      \
  }
#define MVAMG_RESTRICT(KM)          \
  if (narrow) {                     \
    MVAMG_RESTRICT_L(KM, 16)        \
  } else {                          \
    MVAMG_RESTRICT_L(KM, 64)        \
  }
  switch (P.kmax) {
    case 1: MVAMG_RESTRICT(1); break;
    case 2: MVAMG_RESTRICT(2); break;
    case 3:
    case 4: MVAMG_RESTRICT(4); break;
    default: MVAMG_RESTRICT(8); break;
  }
#undef MVAMG_RESTRICT_L
#undef MVAMG_RESTRICT
  LAUNCHCHECK("restrict");
  if (kcyc && next_smoothed)
    kc_fcg2<T>(h, l + 1, rc, xc, smoother, st, true);
  else
    vcycle<T>(h, l + 1, rc, xc, smoother, st, next_smoothed, nullptr, false, kcyc);
  {
    const bool gs = smoother == MVAMG_SMOOTH_GS;
    const int nr = gs ? P.ncut : P.nf;
    const double nu = gs ? (double)P.nu_cut : (double)P.nu;
    const int pg = grid_elem(std::max(nr, 1));
    const double pby = skip_bytes(h, l, nu * sizeof(T) + (double)nr * (4 + 2 * sizeof(T)) + (double)C.n * sizeof(T));
    const Skip sk = lskip(h, l, SKIP_ROW);
    if (nr > 0) switch (P.kmax) {
      case 1: klaunch(h, MVAMG_KC_PROLONG, pby, k_prolong_rows<T, 1>, pg, kBlock, st, nr, P.nf, P.cinfo, tUrow<T>(P), xc, x, sk); break;
      case 2: klaunch(h, MVAMG_KC_PROLONG, pby, k_prolong_rows<T, 2>, pg, kBlock, st, nr, P.nf, P.cinfo, tUrow<T>(P), xc, x, sk); break;
      case 3:
      case 4: klaunch(h, MVAMG_KC_PROLONG, pby, k_prolong_rows<T, 4>, pg, kBlock, st, nr, P.nf, P.cinfo, tUrow<T>(P), xc, x, sk); break;
      default: klaunch(h, MVAMG_KC_PROLONG, pby, k_prolong_rows<T, 8>, pg, kBlock, st, nr, P.nf, P.cinfo, tUrow<T>(P), xc, x, sk); break;
    }
  }
  LAUNCHCHECK("prolong");
  // post-smoothing: one backward sweep
  if (smoother == MVAMG_SMOOTH_GS) {
    int off = 0;
    for (int c = L.ns - 1; c >= 0; --c) off += gs_stage<T>(h, l, L, c, r, x, 1, st, false, dot_part ? dot_part + off : nullptr);
    if (dot_part) h->dot_nparts = off;
  } else {
    resid<T, 0>(h, l, L, r, x, s, M_NONE, st);
    k_l1_update<T><<<grid_for(L.n), kBlock, 0, st>>>(L.n, ldl1<T>(L), s, x);
  }
  LAUNCHCHECK("vcycle");
}

// y ~ A_m^{-1} g: two flexible-CG iterations from y = 0 on level m (not the
// finest, not the coarsest), each preconditioned by the K-cycle of level m.
// y is the level's x vector (c1 is built there); y_started: the restriction
// that produced g has already taken the first smoothing step of c1.
template <>
void kc_fcg2<double>(mvamg_hier* h, int m, const double* g, double* y, int smoother, hipStream_t st, bool y_started) {
  DevLevel& L = h->lv[m];
  const int n = L.n, grid = std::min(grid_for(n), 512);
  // c1 = K g, v1 = A c1, (c1.v1, c1.g), r2 = g - alpha1 v1
  vcycle<double>(h, m, g, y, smoother, st, y_started, nullptr, false, true);
  resid<double, 2>(h, m, L, nullptr, y, L.kv1, M_NONE, st);
  k_kdots<2><<<grid, kBlock, 0, st>>>(n, y, L.kv1, y, g, nullptr, nullptr, h->part);
  k_kfinish<2><<<1, kBlock, 0, st>>>(grid, h->part, L.ks);
  k_kresid<<<grid_elem(n), kBlock, 0, st>>>(n, L.ks, g, L.kv1, L.kr2);
  // c2 = K r2, v2 = A c2, (c2.v1, c2.v2, c2.r2), y = combination of c1, c2
  vcycle<double>(h, m, L.kr2, L.kc2, smoother, st, false, nullptr, false, true);
  resid<double, 2>(h, m, L, nullptr, L.kc2, L.kv2, M_NONE, st);
  k_kdots<3><<<grid, kBlock, 0, st>>>(n, L.kc2, L.kv1, L.kc2, L.kv2, L.kc2, L.kr2, h->part);
  k_kfinish<3><<<1, kBlock, 0, st>>>(grid, h->part, L.ks + 2);
  k_kcombine<<<grid_elem(n), kBlock, 0, st>>>(n, L.ks, y, L.kc2, y);
  LAUNCHCHECK("kc_fcg2");
}

template <>
void kc_fcg2<float>(mvamg_hier*, int, const float*, float*, int, hipStream_t, bool) {
  throw Error(MVAMG_ERR_ARG, "the K-cycle runs in binary64 only");
}

// z = B r for level-0 binary64 vectors in smoother order (the K-cycle when
// cycle is MVAMG_CYCLE_K)
void apply_B(mvamg_hier* h, const double* r, double* z, int precision, int smoother, hipStream_t st,
             int cycle = MVAMG_CYCLE_V) {
  if (cycle == MVAMG_CYCLE_K) {
    if (precision != 64) throw Error(MVAMG_ERR_ARG, "the K-cycle runs in binary64 only");
    vcycle<double>(h, 0, r, z, smoother, st, false, nullptr, false, true);
  } else if (precision == 64) {
    vcycle<double>(h, 0, r, z, smoother, st);
  } else {
    DevLevel& L = h->lv[0];
    k_cast<double, float><<<grid_for(L.n), kBlock, 0, st>>>(L.n, r, L.r32);
    vcycle<float>(h, 0, L.r32, L.x32, smoother, st);
    k_cast<float, double><<<grid_for(L.n), kBlock, 0, st>>>(L.n, L.x32, z);
    LAUNCHCHECK("apply_B32");
  }
}

// q = A p (level 0, smoother order) with p.q into S_PQ / alpha
void spmv0_dot(mvamg_hier* h, const double* p, double* q, int mode, hipStream_t st) {
  resid<double, 1>(h, 0, h->lv[0], nullptr, p, q, mode, st);
}

void dot(mvamg_hier* h, const double* a, const double* b, int mode, hipStream_t st) {
  const int n = h->n;
  k_dot<1><<<grid_for(n), kBlock, 0, st>>>(n, a, b, nullptr, nullptr, mkred(h));
  LAUNCHCHECK("dot");
  finish(h, 1, grid_for(n), mode, st);
}

void read_scalars(mvamg_hier* h, hipStream_t st) {
  HIPCHECK(hipMemcpyAsync(h->pinned, h->scal, S_NSCAL * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
}

void fill_level_values(mvamg_hier* h, int l, const double* val_file, hipStream_t st) {
  DevLevel& L = h->lv[l];
  L.vcoded = L.dcoded = false;  // the codes describe the values uploaded with the layout
  k_fill_values<<<grid_for(L.nent), kBlock, 0, st>>>(L.nent, L.src, val_file, L.val);
  k_fill_values<<<grid_for(L.ndblk), kBlock, 0, st>>>(L.ndblk, L.dsrc, val_file, L.dblk);
  LAUNCHCHECK("fill_values");
}

void derive_level(mvamg_hier* h, int l, hipStream_t st) {
  DevLevel& L = h->lv[l];
  k_to_f32<<<grid_for(L.nent), kBlock, 0, st>>>(L.nent, L.val, L.val32);
  k_to_f32<<<grid_for(L.ndblk), kBlock, 0, st>>>(L.ndblk, L.dblk, L.dblk32);
  if (L.vcoded) k_to_f32<<<1, kBlock, 0, st>>>(L.nvtab, L.vtab, L.vtab32);
  if (L.dcoded) k_to_f32<<<1, kBlock, 0, st>>>(L.ndtab, L.dtab, L.dtab32);
  if (L.sell) {
    k_l1norm_sell<<<(L.nslabs + 3) / 4, kBlock, 0, st>>>(L.slabs, L.nslabs, L.val, L.dblk, L.dl1);
  } else {
    k_l1norm_grp<<<grid_for(L.ng), kBlock, 0, st>>>(L.ng, L.gstart, L.rowptr, L.val, L.dboff, L.dblk, L.dl1);
  }
  k_to_f32<<<grid_for(L.n), kBlock, 0, st>>>(L.n, L.dl1, L.dl1_32);
  LAUNCHCHECK("derive_level");
}

mvamg_status fail_status(const Error& e) {
  g_err = e.what();
  return (mvamg_status)e.status;
}

// Calls that need the whole batch in one hierarchy
void no_small_path(const mvamg_hier* h) {
  if (h->nmini > 0 || h->nl == 0)
    throw Error(MVAMG_ERR_ARG, "not available on a batch with problems on the small-problem path");
}

void check_device(const mvamg_hier* h) {
  int dev = -1;
  HIPCHECK(hipGetDevice(&dev));
  if (dev != h->device) throw Error(MVAMG_ERR_ARG, "handle used with a different current device");
}

// One CG half-step A: q = A p, alpha = rho / p.q, r -= alpha q, r.r --
// whose finisher also writes the scalars to the mapped host buffer (no copy
// node).  x += alpha p is left pending: the next half-step B applies it
// where it reads p anyway, or pcg after its last step (k_x_update).
// stage0: the update also writes the next cycle's first sweep stage into z
// (see cg_step_b).
void cg_step_a(mvamg_hier* h, hipStream_t st, bool stage0) {
  const int n = h->n, eg = grid_for(n);
  spmv0_dot(h, h->p, h->q, M_PQ, st);
  k_axpy_dot<<<eg, kBlock, 0, st>>>(n, h->scal, h->q, h->r, mkred(h), stage0 ? h->lv[0].rows0 : 0,
                                     svals<double>(h->lv[0]), h->z);
  LAUNCHCHECK("axpy");
  finish(h, 1, eg, M_STORE_RR, st, h->pinned_dev);
}

// Half-step B: z = B r, beta (standard or flexible), the pending x += alpha p,
// p = z + beta p.  In
// binary64 with Gauss-Seidel on a sliced-ELL fine level, the cycle's last
// sweep writes the partials of z.r itself.
// The binary64 Gauss-Seidel cycle on a sliced-ELL fine level: its first
// sweep stage comes with the preceding CG update (cg_step_a).
bool fused_cycle(const mvamg_hier* h, int precision, int smoother, int cycle) {
  return precision == 64 && smoother == MVAMG_SMOOTH_GS && cycle == MVAMG_CYCLE_V && h->nl > 1 && h->lv[0].sell;
}

void cg_step_b(mvamg_hier* h, int precision, int smoother, int cycle, hipStream_t st) {
  const int n = h->n, eg = grid_for(n);
  if (fused_cycle(h, precision, smoother, cycle)) {
    vcycle<double>(h, 0, h->r, h->z, smoother, st, false, h->part, true);
    finish(h, 1, h->dot_nparts, M_RZ, st);
  } else if (precision == 32 || cycle == MVAMG_CYCLE_K) {
    // a preconditioner that is not a fixed symmetric operator: flexible beta
    apply_B(h, h->r, h->z, precision, smoother, st, cycle);
    k_dot<2><<<eg, kBlock, 0, st>>>(n, h->z, h->r, h->z, h->q, mkred(h));
    finish(h, 2, eg, M_RZ_FLEX, st);
  } else {
    apply_B(h, h->r, h->z, precision, smoother, st);
    k_dot<1><<<eg, kBlock, 0, st>>>(n, h->z, h->r, nullptr, nullptr, mkred(h));
    finish(h, 1, eg, M_RZ, st);
  }
  k_xpay<<<grid_elem(n), kBlock, 0, st>>>(n, h->scal, h->z, h->p, h->x);
  LAUNCHCHECK("xpay");
}

// One full iteration (B then A) captured once as a HIP graph and replayed:
// about 60 kernels per launch instead of as many host launches.
hipGraphExec_t iteration_graph(mvamg_hier* h, int precision, int smoother, int cycle) {
  const int key = (precision * 4 + smoother) * 2 + cycle;
  auto it = h->graphs.find(key);
  if (it != h->graphs.end()) return it->second;
  if (!h->cap) HIPCHECK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  HIPCHECK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  try {
    cg_step_b(h, precision, smoother, cycle, h->cap);
    cg_step_a(h, h->cap, fused_cycle(h, precision, smoother, cycle));
  } catch (...) {
    (void)hipStreamEndCapture(h->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIPCHECK(hipStreamEndCapture(h->cap, &g));
  hipGraphExec_t ge = nullptr;
  const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  hipcheck(e, "hipGraphInstantiate");
  h->graphs[key] = ge;
  return ge;
}

// Captured iteration graphs are rebuilt on the next solve.
void drop_graphs(mvamg_hier* h) {
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.second);
  h->graphs.clear();
}

// Level-0 values replaced by val (file CSR order, nnz entries): a near-by
// matrix with the hierarchy's pattern.  Drops the value codes (the kernels
// read the values from now on) and the captured iterations that hold them.
void refill_fine(mvamg_hier* h, const double* val, hipStream_t st) {
  const bool coded = h->lv[0].vcoded || h->lv[0].dcoded;
  fill_level_values(h, 0, val, st);
  derive_level(h, 0, st);
  k_copy<double><<<grid_for(h->nnz), kBlock, 0, st>>>((int)h->nnz, val, h->fval);
  LAUNCHCHECK("refill_fine");
  if (coded) drop_graphs(h);
}

// The matrix a solve is asked for.  rowptr/col (both or neither): checked
// against the hierarchy's level-0 pattern; val: compared with the values in
// use and, where any differs, taken as the new level-0 values.
void use_matrix(mvamg_hier* h, const int* rowptr, const int* col, const double* val, hipStream_t st) {
  if ((rowptr == nullptr) != (col == nullptr)) throw Error(MVAMG_ERR_ARG, "rowptr and col are passed together");
  if (!rowptr && !val) return;
  k_fill<int><<<1, kBlock, 0, st>>>(2, 0, h->cmpflag);
  if (rowptr) {
    k_differs<int><<<grid_for(h->n + 1), kBlock, 0, st>>>(h->n + 1, rowptr, h->frp, h->cmpflag);
    k_differs<int><<<grid_for(h->nnz), kBlock, 0, st>>>(h->nnz, col, h->fci, h->cmpflag);
  }
  if (val) k_differs<double><<<grid_for(h->nnz), kBlock, 0, st>>>(h->nnz, val, h->fval, h->cmpflag + 1);
  LAUNCHCHECK("use_matrix");
  int flags[2] = {0, 0};
  HIPCHECK(hipMemcpyAsync(flags, h->cmpflag, sizeof(flags), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  if (flags[0]) throw Error(MVAMG_ERR_ARG, "matrix pattern differs from the hierarchy's finest level");
  if (flags[1]) refill_fine(h, val, st);
}

// Core CG loop shared by solve and adjoint solve.
mvamg_status pcg(mvamg_hier* h, const double* b_file, double* x_file, const mvamg_solve_params* prm,
                 mvamg_info* info, hipStream_t st) {
  if (!prm || !b_file || !x_file) throw Error(MVAMG_ERR_ARG, "null argument");
  if (prm->precision != 64 && prm->precision != 32) throw Error(MVAMG_ERR_ARG, "precision must be 64 or 32");
  if (prm->smoother != MVAMG_SMOOTH_GS && prm->smoother != MVAMG_SMOOTH_L1JACOBI)
    throw Error(MVAMG_ERR_ARG, "unknown smoother");
  if (prm->cycle != MVAMG_CYCLE_V && prm->cycle != MVAMG_CYCLE_K) throw Error(MVAMG_ERR_ARG, "unknown cycle");
  if (prm->cycle == MVAMG_CYCLE_K && prm->precision != 64)
    throw Error(MVAMG_ERR_ARG, "the K-cycle runs in binary64 only");
  if (prm->maxit < 0 || !(prm->rtol >= 0.0)) throw Error(MVAMG_ERR_ARG, "invalid maxit or rtol");
  if (h->nprob > 0 || h->nall > 0) throw Error(MVAMG_ERR_ARG, "a batch handle is solved with mvamg_batch_pcg_solve");
  check_device(h);
  const int n = h->n;
  const int eg = grid_for(n);
  DevLevel& L0 = h->lv[0];
  mvamg_info inf{};
  const bool flex = (prm->precision == 32);
  // into smoother order
  k_gather<<<eg, kBlock, 0, st>>>(n, h->perm0, b_file, h->b);
  k_gather<<<eg, kBlock, 0, st>>>(n, h->perm0, x_file, h->x);
  LAUNCHCHECK("gather");
  HIPCHECK(hipMemsetAsync(h->scal, 0, S_NSCAL * sizeof(double), st));
  resid<double, 0>(h, 0, L0, h->b, h->x, h->r, M_NONE, st);
  dot(h, h->r, h->r, M_STORE_R0, st);
  read_scalars(h, st);
  const double r0 = std::sqrt(h->pinned[S_R0]);
  if (!std::isfinite(r0)) throw Error(MVAMG_ERR_NONFINITE, "non-finite initial residual (check b and x0)");
  if (prm->history) prm->history[0] = 1.0;
  mvamg_status status = MVAMG_NOT_CONVERGED;
  double h_last = 1.0;
  int64_t steps = 0;  // CG steps queued in this solve (the device counts them in scal[S_STEPS])
  if (r0 == 0.0) {
    status = MVAMG_OK;
    inf.converged = 1;
    h_last = 0.0;
  } else {
    int it = 0;
    const int max_restarts = flex ? std::max(0, prm->max_restarts) : 0;
    for (int restart = 0; restart <= max_restarts && it < prm->maxit; ++restart) {
      if (restart > 0) {
        resid<double, 0>(h, 0, L0, h->b, h->x, h->r, M_NONE, st);
        inf.restarts = restart;
      }
      apply_B(h, h->r, h->z, prm->precision, prm->smoother, st, prm->cycle);
      dot(h, h->r, h->z, M_RHO0, st);
      k_copy<double><<<eg, kBlock, 0, st>>>(n, h->z, h->p);
      bool met = false;
      hipGraphExec_t ge =
          (h->use_graphs && !h->prof) ? iteration_graph(h, prm->precision, prm->smoother, prm->cycle) : nullptr;
      // With the iteration graph the device runs one iteration ahead of the
      // host: iteration j + 1 is queued before j's scalars are read (they sit
      // in host slot j mod 2, see k_finish), so the device never waits for
      // the host between iterations.  An iteration queued past the one that
      // stops the loop is discarded; its only lasting effect is the pending
      // x += alpha p of the stopping step, applied by its p update with the
      // same arithmetic as k_x_update.
      if (ge && !h->itev[0])
        for (hipEvent_t& e : h->itev) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      bool first = true;
      int queued = it;  // iterations queued; it: iterations whose scalars were read
      auto queue_next = [&]() {
        if (first) {
          cg_step_a(h, st, fused_cycle(h, prm->precision, prm->smoother, prm->cycle));
          first = false;
        } else if (ge) {
          HIPCHECK(hipGraphLaunch(ge, st));
        } else {
          cg_step_b(h, prm->precision, prm->smoother, prm->cycle, st);
          cg_step_a(h, st, fused_cycle(h, prm->precision, prm->smoother, prm->cycle));
        }
        if (ge) HIPCHECK(hipEventRecord(h->itev[steps & 1], st));
        ++steps;
        ++queued;
      };
      while (it < prm->maxit) {
        if (queued == it) queue_next();
        const int64_t rd = steps - (queued - it);  // step index of iteration it + 1
        if (ge && queued < prm->maxit) queue_next();
        if (ge)
          HIPCHECK(hipEventSynchronize(h->itev[rd & 1]));
        else
          HIPCHECK(hipStreamSynchronize(st));
        ++it;
        const double* sc = h->pinned + (rd & 1) * S_NSCAL;
        if (sc[S_FLAG] != 0.0) {
          inf.iterations = it;
          (void)hipStreamSynchronize(st);
          throw Error(MVAMG_ERR_BREAKDOWN, "CG breakdown: p^T A p <= 0 (matrix not s.p.d.)");
        }
        h_last = std::sqrt(sc[S_RR]) / r0;
        if (prm->history) prm->history[it] = h_last;
        if (!std::isfinite(h_last)) {
          (void)hipStreamSynchronize(st);
          throw Error(MVAMG_ERR_NONFINITE, "non-finite residual during CG");
        }
        if (h_last <= prm->rtol) {
          met = true;
          break;
        }
      }
      // the last step's pending x += alpha p (see cg_step_a), unless a
      // discarded iteration has applied it
      if (!first && queued == it) {
        k_x_update<<<grid_elem(n), kBlock, 0, st>>>(n, h->scal, h->p, h->x);
        LAUNCHCHECK("x_update");
      }
      if (!flex) {
        if (met) status = MVAMG_OK;
        break;
      }
      // binary32 cycle: confirm with the true residual in binary64
      resid<double, 0>(h, 0, L0, h->b, h->x, h->q, M_NONE, st);
      dot(h, h->q, h->q, M_STORE_RR, st);
      read_scalars(h, st);
      const double tr = std::sqrt(h->pinned[S_RR]) / r0;
      if (met && tr <= prm->rtol) {
        status = MVAMG_OK;
        break;
      }
    }
    inf.iterations = it;
    inf.converged = (status == MVAMG_OK);
  }
  inf.rel_res = h_last;
  // true residual in binary64 and back to file order
  resid<double, 0>(h, 0, L0, h->b, h->x, h->q, M_NONE, st);
  dot(h, h->q, h->q, M_STORE_RR, st);
  k_scatter<<<eg, kBlock, 0, st>>>(n, h->perm0, h->x, x_file);
  LAUNCHCHECK("scatter");
  read_scalars(h, st);
  inf.rel_res_true = (r0 > 0.0) ? std::sqrt(h->pinned[S_RR]) / r0 : 0.0;
  if (h->prof) harvest(h);
  if (info) *info = inf;
  return status;
}

// Dense Cholesky of one coarsest block (CSR C padded with the identity to np
// rows) and its inverse L^{-T} L^{-1} written to out (np x np).  M and Li are
// scratch of at least np x np; the block's CSR arrays are added to temps.
void factor_block(mvamg_hier* h, const HostLevel& C, int np, double* M, double* Li, double* out, int* flag,
                  std::vector<void*>& temps, hipStream_t st) {
  const int nb = np / TD;
  int* rp = h->upload_vec(C.rp, st);
  int* ci = h->upload_vec(C.ci, st);
  double* v = h->upload_vec(C.v, st);
  temps.push_back(rp);
  temps.push_back(ci);
  temps.push_back(v);
  HIPCHECK(hipMemsetAsync(M, 0, sizeof(double) * (size_t)np * np, st));
  k_csr_to_padded<<<grid_for(np), kBlock, 0, st>>>(C.n, np, rp, ci, v, M);
  for (int kb = 0; kb < nb; ++kb) {
    k_potrf_tile<<<1, 256, 0, st>>>(M, np, kb, flag);
    const int m = nb - kb - 1;
    if (m > 0) {
      k_trsm_tile<<<m, 256, 0, st>>>(M, np, kb);
      k_update_tiles<<<dim3(m, m), 256, 0, st>>>(M, np, kb);
    }
  }
  k_trtri_diag<<<nb, 256, 0, st>>>(M, Li, np);
  for (int i = 1; i < nb; ++i) k_trtri_row<<<i, 256, 0, st>>>(M, Li, np, i);
  k_lauum<<<dim3(nb, nb), 256, 0, st>>>(Li, out, np);
  LAUNCHCHECK("factor_block");
}

// Device copy of a hierarchy; cblk lists the diagonal blocks of its
// coarsest level (one for a single problem, one per problem of a batch).
// arena: the caller's device buffer of arena_cap bytes, or null to size
// only (no device work; h->arena_peak is then the bytes an arena needs).
std::unique_ptr<mvamg_hier> upload_hier(const HostHier& H, const std::vector<const HostLevel*>& cblk, hipStream_t st,
                                        const std::vector<int>* rowprob0, void* arena, size_t arena_cap) {
  std::unique_ptr<mvamg_hier> h;
  try {
    if (H.nl < 2) throw Error(MVAMG_ERR_ARG, "hierarchy needs at least two levels");
    if (arena && reinterpret_cast<uintptr_t>(arena) % 256 != 0)
      throw Error(MVAMG_ERR_ARG, "device arena must be 256-byte aligned");
    h.reset(new mvamg_hier);
    h->arena = (unsigned char*)arena;
    h->arena_cap = arena_cap;
    const bool dev = !h->sizing();
    if (dev) HIPCHECK(hipGetDevice(&h->device));
    {
      const char* ev = std::getenv("MVAMG_NO_GRAPH");
      h->use_graphs = !(ev && ev[0] && ev[0] != '0');
    }
    h->nl = H.nl;
    h->n = H.lv[0].n;
    h->nnz = (int64_t)H.lv[0].ci.size();
    for (int l = 0; l < H.nl; ++l) {
      h->lev_n.push_back(H.lv[l].n);
      h->lev_nnz.push_back((int64_t)H.lv[l].ci.size());
    }
    // ---- layouts
    std::vector<LevelLayout> Y(H.nl - 1);
    for (int l = 0; l + 1 < H.nl; ++l) build_level_layout(H.lv[l], Y[l], l == 0 ? rowprob0 : nullptr);
    h->lv.resize(H.nl);
    h->tr.resize(H.nl - 1);
    int maxgrid = 2048;
    for (int l = 0; l + 1 < H.nl; ++l) {
      const LevelLayout& y = Y[l];
      DevLevel& L = h->lv[l];
      L.n = y.n;
      L.sell = y.sell;
      L.G = y.G;
      L.G0 = y.G;
      L.gshared = !y.sell && y.all_shared;
      L.ng = (int)y.gstart.size() - 1;
      L.ns = (int)y.sgrp.size() - 1;
      L.h_sgrp = y.sgrp;
      L.h_sslab = y.sslab;
      L.h_srow.resize(y.sgrp.size());
      for (size_t c = 0; c < y.sgrp.size(); ++c) L.h_srow[c] = y.gstart[y.sgrp[c]];
      L.nslabs = (int)y.slabs.size();
      L.rows0 = y.gstart[y.sgrp[1]];
      L.nent = (int64_t)y.val.size();
      L.nnz = (int64_t)H.lv[l].ci.size();
      L.stage_rows.assign(L.ns, 0);
      L.stage_nnz.assign(L.ns, 0);
      for (int c = 0; c < L.ns; ++c)
        for (int p = y.gstart[y.sgrp[c]]; p < y.gstart[y.sgrp[c + 1]]; ++p) {
          const int i = y.perm[p];
          L.stage_rows[c] += 1;
          L.stage_nnz[c] += H.lv[l].rp[i + 1] - H.lv[l].rp[i];
        }
      L.ndblk = (int64_t)y.dblk.size();
      if (y.sell) {
        L.slabs = h->upload_vec(y.slabs, st);
        {
          auto spatial = [&](int q1) {
            std::vector<int> o(q1);
            for (int q = 0; q < q1; ++q) o[q] = q;
            std::stable_sort(o.begin(), o.end(),
                             [&](int a, int b) { return y.perm[y.slabs[a].row0] < y.perm[y.slabs[b].row0]; });
            std::vector<Slab> v(q1);
            for (int q = 0; q < q1; ++q) v[q] = y.slabs[o[q]];
            return v;
          };
          L.nslab_part = y.sslab[L.ns - 1];
          L.bslab_full = h->upload_vec(spatial(L.nslabs), st);
          L.bslab_part = L.nslab_part > 0 ? h->upload_vec(spatial(L.nslab_part), st) : nullptr;
        }
        L.col16 = h->upload_vec(y.col16, st);
        L.pk = h->upload_vec(y.pk, st);
        L.cbase = h->upload_vec(y.cbase.empty() ? std::vector<int>(8, 0) : y.cbase, st);
        L.scb = h->upload_vec(y.scb, st);
        L.nnz16 = y.nnz16;
        if (y.vcoded) {
          L.vcode = h->upload_vec(y.vcode, st);
          L.vtab = h->upload_vec(y.vtab, st);
          L.vtab32 = h->dalloc<float>(y.vtab.size());
          L.nvtab = (int)y.vtab.size();
          L.vcoded = true;
        }
        if (y.dcoded) {
          L.dcode = h->upload_vec(y.dcode, st);
          L.dtab = h->upload_vec(y.dtab, st);
          L.dtab32 = h->dalloc<float>(y.dtab.size());
          L.ndtab = (int)y.dtab.size();
          L.dcoded = true;
        }
        L.stage_nnz16 = y.stage_nnz16;
        L.stage_gidx.assign(L.ns, 0);
        L.stage_later_idx.assign(L.ns, 0);
      } else {
        L.stage_nnz16.assign(L.ns, 0);
        L.stage_gidx = y.stage_gidx;
        L.stage_later_idx = y.stage_later_idx;
        for (int64_t v : y.stage_gidx) L.gidx += v;
      }
      if (!y.sell) {
        L.rowptr = h->upload_vec(y.rowptr, st);
        std::vector<int> rec((size_t)L.ng * kRec, 0);
        for (int g = 0; g < L.ng; ++g) {
          const int p0 = y.gstart[g], k = y.gstart[g + 1] - p0;
          int* R = &rec[(size_t)g * kRec];
          R[0] = p0;
          R[1] = k;
          R[2] = y.dboff[g];
          for (int q = 0; q <= kKmax; ++q) R[3 + q] = y.rowptr[p0 + std::min(q, k)];
          for (int q = 0; q < kKmax; ++q) R[12 + q] = q < k ? y.rsplit[p0 + q] : y.rowptr[p0 + k];
          R[20] = y.gcsh[g];
          R[21] = y.gcm[g];
        }
        L.gcol = h->upload_vec(y.gcol.empty() ? std::vector<int>(1, 0) : y.gcol, st);
        // entries of later stages, per stage (not read by the forward sweep from zero)
        L.stage_later.assign(L.ns, 0);
        for (int c = 0; c < L.ns; ++c)
          for (int p = y.gstart[y.sgrp[c]]; p < y.gstart[y.sgrp[c + 1]]; ++p) L.stage_later[c] += y.rowptr[p + 1] - y.rsplit[p];
        L.rec = h->upload_vec(rec, st);
      }
      L.col = h->upload_vec(y.col, st);
      L.val = h->upload_vec(y.val, st);
      L.val32 = h->dalloc<float>(y.val.size());
      L.gstart = h->upload_vec(y.gstart, st);
      L.dboff = h->upload_vec(y.dboff, st);
      L.dblk = h->upload_vec(y.dblk, st);
      L.dblk32 = h->dalloc<float>(y.dblk.size());
      if (l == 0) {
        L.src = h->upload_vec(y.src, st);
        L.dsrc = h->upload_vec(y.dsrc, st);
      }
      L.dl1 = h->dalloc<double>(y.n);
      L.dl1_32 = h->dalloc<float>(y.n);
      L.s = h->dalloc<double>(y.n);
      L.s32 = h->dalloc<float>(y.n);
      L.r32 = h->dalloc<float>(y.n);
      L.x32 = h->dalloc<float>(y.n);
      if (l > 0) {
        L.r = h->dalloc<double>(y.n);
        L.x = h->dalloc<double>(y.n);
        L.kv1 = h->dalloc<double>(y.n);
        L.kr2 = h->dalloc<double>(y.n);
        L.kc2 = h->dalloc<double>(y.n);
        L.kv2 = h->dalloc<double>(y.n);
        L.ks = h->dalloc<double>(8);
      }
      maxgrid = std::max(maxgrid, resid_grid(L));
    }
    for (int l = 0; l + 1 < H.nl; ++l) {
      TransferLayout T;
      build_transfer_layout(H.lv[l], Y[l], (l + 2 < H.nl) ? &Y[l + 1] : nullptr, T);
      DevTransfer& P = h->tr[l];
      P.nagg = T.nagg;
      P.nu = (int64_t)T.U.size();
      P.arows = h->upload_vec(T.arows, st);
      {
        // per-aggregate records; when level l+1 is smoothed, the coarse rows
        // cst[a] .. cst[a] + k - 1 must be one of its smoother groups
        std::vector<int> rec((size_t)T.nagg * kARec, 0);
        for (int a = 0; a < T.nagg; ++a) {
          int* R = rec.data() + (size_t)a * kARec;
          R[AR_M0] = T.aptr[a];
          R[AR_NA] = T.aptr[a + 1] - T.aptr[a];
          R[AR_K] = T.kk[a];
          R[AR_UOFF] = T.uoff[a];
          R[AR_C0] = T.cst[a];
          R[AR_DB] = -1;
        }
        if (l + 2 < H.nl) {
          const LevelLayout& yc = Y[l + 1];
          std::vector<int> rowgrp(yc.n);
          for (int g = 0; g + 1 < (int)yc.gstart.size(); ++g)
            for (int p = yc.gstart[g]; p < yc.gstart[g + 1]; ++p) rowgrp[p] = g;
          for (int a = 0; a < T.nagg; ++a) {
            const int g = rowgrp[T.cst[a]];
            if (yc.gstart[g] != T.cst[a] || yc.gstart[g + 1] - yc.gstart[g] != T.kk[a])
              throw Error(MVAMG_ERR_FILE, "coarse dofs of an aggregate are not one smoother group");
            if (g < yc.sgrp[1]) rec[(size_t)a * kARec + AR_DB] = yc.dboff[g];
          }
        }
        P.arec = h->upload_vec(rec, st);
      }
      P.U = h->upload_vec(T.U, st);
      P.U32 = h->dalloc<float>(T.U.size());
      if (dev) {
        k_to_f32<<<grid_for((int64_t)T.U.size()), kBlock, 0, st>>>((int64_t)T.U.size(), P.U, P.U32);
        LAUNCHCHECK("U32");
      }
      {
        // row-order copy of P for the prolongation
        const int nf = H.lv[l].n;
        int kmax = 1;
        for (int a = 0; a < T.nagg; ++a) kmax = std::max(kmax, T.kk[a]);
        if (kmax > kKmax) throw Error(MVAMG_ERR_ARG, "aggregate basis wider than 8 columns is not supported");
        // the prolongation kernels read all planes of their instantiation
        // (kmax rounded up to 1, 2, 4 or 8); planes past an aggregate's k are zero
        const int kpad = kmax <= 1 ? 1 : kmax <= 2 ? 2 : kmax <= 4 ? 4 : 8;
        std::vector<int> cinfo(nf);
        std::vector<double> urow((size_t)kpad * nf, 0.0);
        for (int a = 0; a < T.nagg; ++a) {
          const int m = T.aptr[a + 1] - T.aptr[a], k = T.kk[a];
          if ((int64_t)T.cst[a] * 8 >= ((int64_t)1 << 31)) throw Error(MVAMG_ERR_ARG, "coarse level too large");
          for (int li = 0; li < m; ++li) {
            const int p = T.arows[T.aptr[a] + li];
            cinfo[p] = T.cst[a] * 8 + (k - 1);
            for (int q = 0; q < k; ++q) urow[(size_t)q * nf + p] = T.U[(size_t)T.uoff[a] + (size_t)q * m + li];
          }
        }
        P.nf = nf;
        P.kmax = kmax;
        const LevelLayout& yf = Y[l];
        const int nsf = (int)yf.sgrp.size() - 1;
        const bool point = (int)yf.gstart.size() - 1 == nf;
        P.ncut = point ? yf.gstart[yf.sgrp[nsf - 1]] : nf;
        P.nu_cut = 0;
        for (int p = 0; p < P.ncut; ++p) P.nu_cut += (cinfo[p] & 7) + 1;
        P.nu_scut = P.nu_cut;
        P.cinfo = h->upload_vec(cinfo, st);
        P.Urow = h->upload_vec(urow, st);
        P.Urow32 = h->dalloc<float>(urow.size());
        if (dev) {
          k_to_f32<<<grid_for((int64_t)urow.size()), kBlock, 0, st>>>((int64_t)urow.size(), P.Urow, P.Urow32);
          LAUNCHCHECK("Urow32");
        }
      }
    }
    // ---- coarsest level: blocked dense Cholesky and inverse of every diagonal block
    {
      const HostLevel& C = H.lv[H.nl - 1];
      DevLevel& LC = h->lv[H.nl - 1];
      LC.n = C.n;
      LC.r = h->dalloc<double>(C.n);
      LC.x = h->dalloc<double>(C.n);
      LC.r32 = h->dalloc<float>(C.n);
      LC.x32 = h->dalloc<float>(C.n);
      DevCoarse& D = h->co;
      D.n = C.n;
      D.nb = (int)cblk.size();
      std::vector<int> coff(D.nb + 1, 0), cnp(D.nb);
      std::vector<int64_t> aoff(D.nb + 1, 0);
      int npmax = 0;
      for (int bk = 0; bk < D.nb; ++bk) {
        const int nbk = cblk[bk]->n;
        cnp[bk] = ((nbk + TD - 1) / TD) * TD;
        if ((int64_t)cnp[bk] * cnp[bk] > ((int64_t)1 << 29))
          throw Error(MVAMG_ERR_ARG, "coarsest level too large for a dense solve");
        coff[bk + 1] = coff[bk] + nbk;
        aoff[bk + 1] = aoff[bk] + (int64_t)cnp[bk] * cnp[bk];
        npmax = std::max(npmax, cnp[bk]);
        D.ainv_entries += (double)nbk * nbk;
      }
      if (coff[D.nb] != C.n) throw Error(MVAMG_ERR_ARG, "coarsest blocks do not cover the coarsest level");
      D.np = cnp[0];
      D.r = h->dalloc<double>(C.n);
      D.z = h->dalloc<double>(C.n);
      D.Ainv = h->dalloc<double>((size_t)aoff[D.nb]);
      double* M = h->dalloc<double>((size_t)npmax * npmax);
      double* Li = h->dalloc<double>((size_t)npmax * npmax);
      int* flag = h->dalloc<int>(1);
      std::vector<void*> temps;
      if (dev) {
        k_fill<int><<<1, kBlock, 0, st>>>(1, 0, flag);
        for (int bk = 0; bk < D.nb; ++bk)
          factor_block(h.get(), *cblk[bk], cnp[bk], M, Li, D.Ainv + aoff[bk], flag, temps, st);
        LAUNCHCHECK("coarsest factorisation");
        int hflag = 0;
        HIPCHECK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        if (hflag) throw Error(MVAMG_ERR_NOT_SPD, "coarsest matrix is not positive definite (Cholesky pivot <= 0)");
      } else {
        // the temporaries factor_block takes: the block's CSR arrays
        for (int bk = 0; bk < D.nb; ++bk) {
          temps.push_back(h->dalloc<int>(cblk[bk]->rp.size()));
          temps.push_back(h->dalloc<int>(cblk[bk]->ci.size()));
          temps.push_back(h->dalloc<double>(cblk[bk]->v.size()));
        }
      }
      // released newest first, so their space is reused by what follows
      for (auto it = temps.rbegin(); it != temps.rend(); ++it) h->dfree(*it);
      h->dfree(flag);
      h->dfree(Li);
      h->dfree(M);
      if (D.nb == 1) {
        D.nt = D.np / 64;
        D.ntiles = D.nt * (D.nt + 1) / 2;
        std::vector<int> tij(2 * (size_t)D.ntiles);
        int t = 0;
        for (int I = 0; I < D.nt; ++I)
          for (int J = 0; J <= I; ++J, ++t) {
            tij[2 * t] = I;
            tij[2 * t + 1] = J;
          }
        D.tij = reinterpret_cast<int2*>(h->upload_vec(tij, st));
        D.tiles = h->dalloc<double>((size_t)D.ntiles * 4096);
        D.spart = h->dalloc<double>((size_t)D.nt * D.nt * 64);
        if (dev) {
          k_pack_tiles<<<D.ntiles, kBlock, 0, st>>>(D.n, D.np, D.tij, D.Ainv, D.tiles);
          LAUNCHCHECK("pack_tiles");
        }
      }
      if (D.nb > 1) {
        std::vector<int> cprob(C.n);
        for (int bk = 0; bk < D.nb; ++bk)
          for (int i = coff[bk]; i < coff[bk + 1]; ++i) cprob[i] = bk;
        D.cprob = h->upload_vec(cprob, st);
        D.coff = h->upload_vec(coff, st);
        D.cnp = h->upload_vec(cnp, st);
        D.aoff = h->upload_vec(aoff, st);
      }
    }
    // ---- batch: problem of every level-0 slab, row and aggregate
    if (rowprob0) {
      const LevelLayout& y = Y[0];
      DevLevel& L0 = h->lv[0];
      std::vector<int> rp(y.n);
      for (int p = 0; p < y.n; ++p) rp[p] = (*rowprob0)[y.perm[p]];
      L0.rowprob = h->upload_vec(rp, st);
      if (y.sell) {
        std::vector<int> sp(y.slabs.size());
        for (size_t q = 0; q < y.slabs.size(); ++q) sp[q] = rp[y.slabs[q].row0];
        L0.slabprob = h->upload_vec(sp, st);
      }
      const HostLevel& F = H.lv[0];
      std::vector<int> ap(F.aptr.size() - 1);
      for (size_t a = 0; a + 1 < F.aptr.size(); ++a) ap[a] = (*rowprob0)[F.arows[F.aptr[a]]];
      h->tr[0].aprob = h->upload_vec(ap, st);
    }
    // ---- level-0 extras and CG state
    {
      const int n = h->n;
      h->perm0 = h->upload_vec(Y[0].perm, st);
      h->iperm0 = h->upload_vec(Y[0].iperm, st);
      h->frp = h->upload_vec(H.lv[0].rp, st);
      h->fci = h->upload_vec(H.lv[0].ci, st);
      h->fval = h->upload_vec(H.lv[0].v, st);
      h->cmpflag = h->dalloc<int>(2);
      h->b = h->dalloc<double>(n);
      h->x = h->dalloc<double>(n);
      h->r = h->dalloc<double>(n);
      h->z = h->dalloc<double>(n);
      h->p = h->dalloc<double>(n);
      h->q = h->dalloc<double>(n);
      h->lv[0].r = h->r;
      h->lv[0].x = h->z;
      h->scal = h->dalloc<double>(S_NSCAL);
      {
        // partials: two values per block of the widest reduction, or the
        // per-stage blocks of the fine backward sweep, whichever is more
        int64_t cap = 2 * (int64_t)maxgrid;
        const DevLevel& F = h->lv[0];
        if (F.sell && F.ns > 0) {
          int64_t d = 0;
          for (int c = 0; c < F.ns; ++c) d += (F.h_sslab[c + 1] - F.h_sslab[c] + 3) / 4;
          cap = std::max(cap, d);
        }
        h->part = h->dalloc<double>((size_t)cap);
      }
      if (dev) {
        HIPCHECK(hipMemsetAsync(h->scal, 0, S_NSCAL * sizeof(double), st));
        // mapped and coherent: a finisher kernel writes it, the host reads it after the stream
        HIPCHECK(hipHostMalloc((void**)&h->pinned, 2 * S_NSCAL * sizeof(double),
                               hipHostMallocMapped | hipHostMallocCoherent));
        HIPCHECK(hipHostGetDevicePointer((void**)&h->pinned_dev, h->pinned, 0));
      }
    }
    if (dev) {
      for (int l = 0; l + 1 < H.nl; ++l) derive_level(h.get(), l, st);
      HIPCHECK(hipStreamSynchronize(st));
    }
  } catch (...) {
    (void)hipStreamSynchronize(st);  // queued work may still use h's memory
    throw;
  }
  return h;
}


#include "multi_host.hpp"
#include "tune_host.hpp"
#include "composite_host.hpp"
#include "setup_host.hpp"
#include "mini_host.hpp"

}  // namespace

// ------------------------------------------- cycle without allocation
//
// Work space of mvamg_cycle_apply_noalloc: one array per device, held until
// the process ends.  Host code never uses the symbol itself as an address
// (on the host it names a stand-in, not device memory); it uses the address
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[MVAMG_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_ptr;  // device -> address of its scratch array

unsigned char* scratch_address(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  HIPCHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) throw Error(MVAMG_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
  g_scratch_ptr[device] = (unsigned char*)ptr;
  return (unsigned char*)ptr;
}

// Carves the work vectors of one cycle (level-0 input and output in smoother
// order, every level's r, x, s in the cycle's precision, the coarsest
// solve's vectors and product slots) out of `base`, or only counts their
// bytes when base is null.  Swaps them into the handle for the lifetime of
// the object and restores the handle's own vectors afterwards.
class ScratchWork {
 public:
  ScratchWork(mvamg_hier* h, int precision, unsigned char* base) : h_(h), base_(base) {
    saved_ = snapshot();
    take(h->r, h->n);
    take(h->z, h->n);
    h->lv[0].r = h->r;
    h->lv[0].x = h->z;
    for (int l = 0; l < h->nl; ++l) {
      DevLevel& L = h->lv[l];
      const bool coarsest = (l == h->nl - 1);
      if (precision == 64) {
        if (!coarsest) take(L.s, L.n);
        if (l > 0) {
          take(L.r, L.n);
          take(L.x, L.n);
        }
      } else {
        if (!coarsest) take(L.s32, L.n);
        take(L.r32, L.n);
        take(L.x32, L.n);
      }
    }
    if (precision == 32) {
      take(h->co.r, h->co.n);
      take(h->co.z, h->co.n);
    }
    if (h->co.nb == 1) take(h->co.spart, (size_t)h->co.nt * h->co.nt * 64);
    if (!base_) restore();
  }
  ~ScratchWork() {
    if (base_) restore();
  }
  size_t bytes() const { return used_; }

 private:
  struct Saved {
    double *hr, *hz;
    std::vector<double*> r, x, s;
    std::vector<float*> r32, x32, s32;
    double *cr, *cz, *spart;
  };
  Saved snapshot() const {
    Saved v{h_->r, h_->z, {}, {}, {}, {}, {}, {}, h_->co.r, h_->co.z, h_->co.spart};
    for (const DevLevel& L : h_->lv) {
      v.r.push_back(L.r);
      v.x.push_back(L.x);
      v.s.push_back(L.s);
      v.r32.push_back(L.r32);
      v.x32.push_back(L.x32);
      v.s32.push_back(L.s32);
    }
    return v;
  }
  void restore() {
    h_->r = saved_.hr;
    h_->z = saved_.hz;
    for (size_t l = 0; l < h_->lv.size(); ++l) {
      DevLevel& L = h_->lv[l];
      L.r = saved_.r[l];
      L.x = saved_.x[l];
      L.s = saved_.s[l];
      L.r32 = saved_.r32[l];
      L.x32 = saved_.x32[l];
      L.s32 = saved_.s32[l];
    }
    h_->co.r = saved_.cr;
    h_->co.z = saved_.cz;
    h_->co.spart = saved_.spart;
  }
  template <typename T>
  void take(T*& slot, size_t count) {
    const size_t at = used_;
    used_ += ((count * sizeof(T) + 255) / 256) * 256;
    if (base_) slot = reinterpret_cast<T*>(base_ + at);
  }
  mvamg_hier* h_;
  unsigned char* base_;
  size_t used_ = 0;
  Saved saved_;
};

}  // namespace

namespace {

// Uploads (or, with a null arena, sizes) a batch.  Problems with at most
// mini_rows rows, and problems whose level count differs from that of the
// most common one among the others, take the one-launch small-problem path
// (mini_kernels.hpp); the rest form one block-diagonal hierarchy solved by
// lockstep launches.
std::unique_ptr<mvamg_hier> upload_batch(const mvamg_hier_host* const* hs, int nprob, int mini_rows, hipStream_t st,
                                         void* arena, size_t arena_bytes) {
  if (!hs || nprob < 1) throw Error(MVAMG_ERR_ARG, "null argument or empty batch");
  if (mini_rows < 0) throw Error(MVAMG_ERR_ARG, "negative small-problem threshold");
  std::vector<const HostHier*> all;
  for (int p = 0; p < nprob; ++p) {
    if (!hs[p]) throw Error(MVAMG_ERR_ARG, "null hierarchy in batch");
    all.push_back(&hs[p]->h);
  }
  // the lockstep part: the problems above the threshold with the most common depth
  std::map<int, int> depth;
  for (const HostHier* H : all)
    if (H->lv[0].n > mini_rows) depth[H->nl]++;
  int dstar = -1, best = 0;
  for (auto& d : depth)
    if (d.second > best) {
      best = d.second;
      dstar = d.first;
    }
  std::vector<int> uid, mid;
  for (int p = 0; p < nprob; ++p) (all[p]->lv[0].n > mini_rows && all[p]->nl == dstar ? uid : mid).push_back(p);
  std::vector<int> aoff(nprob + 1, 0);
  for (int p = 0; p < nprob; ++p) aoff[p + 1] = aoff[p] + all[p]->lv[0].n;
  std::unique_ptr<mvamg_hier> h;
  if (!uid.empty()) {
    std::vector<const HostHier*> Hs;
    for (int p : uid) Hs.push_back(all[p]);
    const HostHier U = union_hierarchy(Hs);
    if (U.nl < 2) throw Error(MVAMG_ERR_ARG, "hierarchy needs at least two levels");
    std::vector<const HostLevel*> cb;
    for (const HostHier* H : Hs) cb.push_back(&H->lv[H->nl - 1]);
    std::vector<int> rowprob0;
    for (size_t q = 0; q < Hs.size(); ++q) rowprob0.insert(rowprob0.end(), Hs[q]->lv[0].n, (int)q);
    h = upload_hier(U, cb, st, &rowprob0, arena, arena_bytes);
    const int nu = (int)uid.size();
    h->nprob = nu;
    h->h_poff.assign(nu + 1, 0);
    int maxn = 1;
    for (int q = 0; q < nu; ++q) {
      h->h_poff[q + 1] = h->h_poff[q] + Hs[q]->lv[0].n;
      maxn = std::max(maxn, Hs[q]->lv[0].n);
    }
    h->poff = h->upload_vec(h->h_poff, st);
    h->pchunks = std::min(kMaxChunks, std::max(1, (maxn + 2047) / 2048));
    // room for every chunk count the autotuner may choose, so nothing grows later
    ensure_multi(h.get(), nu, kMaxChunks);
    if (!mid.empty()) {
      std::vector<int> umap(h->n);
      for (int q = 0; q < nu; ++q)
        for (int i = h->h_poff[q]; i < h->h_poff[q + 1]; ++i) umap[i] = aoff[uid[q]] + (i - h->h_poff[q]);
      h->umap = h->upload_vec(umap, st);
    }
  } else {
    // every problem on the small path: a handle without levels
    h.reset(new mvamg_hier);
    h->arena = (unsigned char*)arena;
    h->arena_cap = arena_bytes;
    if (arena && reinterpret_cast<uintptr_t>(arena) % 256 != 0)
      throw Error(MVAMG_ERR_ARG, "device arena must be 256-byte aligned");
    if (!h->sizing()) HIPCHECK(hipGetDevice(&h->device));
  }
  h->nall = nprob;
  h->h_aoff = aoff;
  h->uid = uid;
  h->mid = mid;
  if (!mid.empty()) {
    MiniBuild B;
    for (int p : mid) mini_add(B, *all[p], aoff[p]);
    h->nmini = (int)mid.size();
    h->mini_maxit = kMiniMaxIt;
    std::vector<int> pb(B.probs.size() * sizeof(MiniProb) / sizeof(int) + 1);
    std::memcpy(pb.data(), B.probs.data(), B.probs.size() * sizeof(MiniProb));
    std::vector<int> lb(B.levs.size() * sizeof(MiniLevel) / sizeof(int) + 1);
    std::memcpy(lb.data(), B.levs.data(), B.levs.size() * sizeof(MiniLevel));
    h->mprobs = reinterpret_cast<MiniProb*>(h->upload_vec(pb, st));
    h->mlevs = reinterpret_cast<MiniLevel*>(h->upload_vec(lb, st));
    h->mints = h->upload_vec(B.ints, st);
    h->mdbls = h->upload_vec(B.dbls, st);
    h->mwork = h->dalloc<double>((size_t)B.work);
    h->mhist = h->dalloc<double>((size_t)h->nmini * (kMiniMaxIt + 1));
    h->minfo = reinterpret_cast<MiniInfo*>(h->dalloc<double>((size_t)h->nmini * (sizeof(MiniInfo) / sizeof(double) + 1)));
    if (!h->sizing()) {
      HIPCHECK(hipStreamCreateWithFlags(&h->mstream, hipStreamNonBlocking));
      HIPCHECK(hipEventCreateWithFlags(&h->mev[0], hipEventDisableTiming));
      HIPCHECK(hipEventCreateWithFlags(&h->mev[1], hipEventDisableTiming));
    }
  }
  if (!h->sizing()) HIPCHECK(hipStreamSynchronize(st));
  return h;
}

// The small-problem path's solve (prm->precision 64): one launch on the
// handle's second stream, ordered after the work queued on st so far; returns
// after queuing.  mini_collect waits for it and writes the results.
void mini_launch(mvamg_hier* h, const double* b, double* x, const mvamg_solve_params* prm, hipStream_t st) {
  if (prm->maxit > h->mini_maxit) throw Error(MVAMG_ERR_ARG, "small-problem path: maxit above 1000");
  HIPCHECK(hipEventRecord(h->mev[0], st));
  HIPCHECK(hipStreamWaitEvent(h->mstream, h->mev[0], 0));
  const int grid = std::min(h->nmini, 1024);
  k_mini_pcg<<<grid, kMiniBlock, 0, h->mstream>>>(h->nmini, h->mprobs, h->mlevs, h->mints, h->mdbls, h->mwork, b,
                                                    x, prm->rtol, prm->maxit, prm->smoother, h->mhist, h->minfo);
  LAUNCHCHECK("mini_pcg");
  HIPCHECK(hipEventRecord(h->mev[1], h->mstream));
}

// Waits for the small path and writes its problems' info and history (the
// caller's order: problem mid[q]); returns whether all converged.
bool mini_collect(mvamg_hier* h, const mvamg_solve_params* prm, mvamg_info* info, hipStream_t st) {
  HIPCHECK(hipStreamWaitEvent(st, h->mev[1], 0));
  std::vector<MiniInfo> mi(h->nmini);
  HIPCHECK(hipMemcpyAsync(mi.data(), h->minfo, sizeof(MiniInfo) * h->nmini, hipMemcpyDeviceToHost, st));
  std::vector<double> hist;
  if (prm->history) {
    hist.resize((size_t)h->nmini * (h->mini_maxit + 1));
    HIPCHECK(hipMemcpyAsync(hist.data(), h->mhist, sizeof(double) * hist.size(), hipMemcpyDeviceToHost, st));
  }
  HIPCHECK(hipStreamSynchronize(st));
  bool all = true;
  for (int q = 0; q < h->nmini; ++q) {
    const MiniInfo& m = mi[q];
    if (m.status == -5) throw Error(MVAMG_ERR_BREAKDOWN, "CG breakdown: p^T A p <= 0 (matrix not s.p.d.)");
    if (m.status == -4) throw Error(MVAMG_ERR_NONFINITE, "non-finite residual during CG");
    const int p = h->mid[q];
    if (info) {
      info[p].iterations = m.iterations;
      info[p].converged = m.converged;
      info[p].restarts = 0;
      info[p].rel_res = m.rel_res;
      info[p].rel_res_true = m.rel_res_true;
    }
    if (prm->history)
      for (int k = 0; k <= m.iterations; ++k)
        prm->history[(size_t)p * (prm->maxit + 1) + k] = hist[(size_t)q * (h->mini_maxit + 1) + k];
    all = all && m.converged;
  }
  return all;
}

}  // namespace

// ====================================================================== ABI

extern "C" {

const char* mvamg_last_error(void) { return g_err.c_str(); }

mvamg_status mvamg_profile(mvamg_hier* h, int enable) {
  try {
    if (!h) throw Error(MVAMG_ERR_ARG, "null handle");
    HIPCHECK(hipDeviceSynchronize());
    if (enable < 0 || enable > 2) throw Error(MVAMG_ERR_ARG, "enable must be 0, 1 or 2");
    harvest(h);
    h->prof = enable != 0;
    h->book_plain = enable == 2;
    for (int k = 0; k < MVAMG_KC_COUNT; ++k) {
      h->kc_launches[k] = 0;
      h->kc_ms[k] = 0.0;
      h->kc_bytes[k] = 0.0;
    }
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_kernel_stats(mvamg_hier* h, int kclass, int64_t* launches, double* ms, double* bytes) {
  try {
    if (!h || kclass < 0 || kclass >= MVAMG_KC_COUNT) throw Error(MVAMG_ERR_ARG, "bad handle or kernel class");
    HIPCHECK(hipDeviceSynchronize());
    harvest(h);
    if (launches) *launches = h->kc_launches[kclass];
    if (ms) *ms = h->kc_ms[kclass];
    if (bytes) *bytes = h->kc_bytes[kclass];
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_hier_read(const char* path, mvamg_hier_host** out) {
  try {
    if (!path || !out) throw Error(MVAMG_ERR_ARG, "null argument");
    *out = nullptr;
    std::unique_ptr<mvamg_hier_host> h(new mvamg_hier_host);
    h->h = read_hierarchy_file(path);
    *out = h.release();
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  } catch (const std::exception& e) {
    g_err = e.what();
    return MVAMG_ERR_FILE;
  }
}

void mvamg_hier_host_free(mvamg_hier_host* h) { delete h; }

mvamg_status mvamg_hier_host_info(const mvamg_hier_host* h, int* nlevels, int* n, int64_t* nnz) {
  if (!h) {
    g_err = "null handle";
    return MVAMG_ERR_ARG;
  }
  if (nlevels) *nlevels = h->h.nl;
  if (n) *n = h->h.lv[0].n;
  if (nnz) *nnz = (int64_t)h->h.lv[0].ci.size();
  return MVAMG_OK;
}

mvamg_status mvamg_arena_bytes(const mvamg_hier_host* hh, int nrhs, size_t* bytes) {
  try {
    if (!hh || !bytes) throw Error(MVAMG_ERR_ARG, "null argument");
    if (nrhs < 1 || nrhs > MVAMG_BLOCK_MAX) throw Error(MVAMG_ERR_ARG, "nrhs must be in 1..32");
    const HostHier& H = hh->h;
    if (H.nl < 2) throw Error(MVAMG_ERR_ARG, "hierarchy needs at least two levels");
    const std::vector<const HostLevel*> cb{&H.lv[H.nl - 1]};
    std::unique_ptr<mvamg_hier> h = upload_hier(H, cb, nullptr, nullptr, nullptr, 0);
    if (nrhs > 1) ensure_block(h.get());
    *bytes = h->arena_peak;
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  } catch (const std::exception& e) {
    g_err = e.what();
    return MVAMG_ERR_HIP;
  }
}

mvamg_status mvamg_upload(const mvamg_hier_host* hh, void* arena, size_t arena_bytes, void* stream, mvamg_hier** out) {
  hipStream_t st = (hipStream_t)stream;
  try {
    if (!hh || !out || !arena) throw Error(MVAMG_ERR_ARG, "null argument");
    *out = nullptr;
    const HostHier& H = hh->h;
    if (H.nl < 2) throw Error(MVAMG_ERR_ARG, "hierarchy needs at least two levels");
    const std::vector<const HostLevel*> cb{&H.lv[H.nl - 1]};
    *out = upload_hier(H, cb, st, nullptr, arena, arena_bytes).release();
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  } catch (const std::exception& e) {
    g_err = e.what();
    return MVAMG_ERR_HIP;
  }
}

mvamg_status mvamg_batch_arena_bytes(const mvamg_hier_host* const* hs, int nprob, int mini_rows, size_t* bytes) {
  try {
    if (!bytes) throw Error(MVAMG_ERR_ARG, "null argument");
    *bytes = upload_batch(hs, nprob, mini_rows, nullptr, nullptr, 0)->arena_peak;
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  } catch (const std::exception& e) {
    g_err = e.what();
    return MVAMG_ERR_HIP;
  }
}

mvamg_status mvamg_batch_upload(const mvamg_hier_host* const* hs, int nprob, int mini_rows, void* arena,
                                size_t arena_bytes, void* stream, mvamg_hier** out) {
  hipStream_t st = (hipStream_t)stream;
  try {
    if (!out || !arena) throw Error(MVAMG_ERR_ARG, "null argument");
    *out = nullptr;
    *out = upload_batch(hs, nprob, mini_rows, st, arena, arena_bytes).release();
    return MVAMG_OK;
  } catch (const Error& e) {
    if (st) (void)hipStreamSynchronize(st);
    return fail_status(e);
  } catch (const std::exception& e) {
    g_err = e.what();
    return MVAMG_ERR_HIP;
  }
}

mvamg_status mvamg_batch_problems(const mvamg_hier* h, int* nprob, int* offsets) {
  if (!h) {
    g_err = "null handle";
    return MVAMG_ERR_ARG;
  }
  // the caller's view: every problem of the batch, on either path
  const int np = h->nall > 0 ? h->nall : h->nprob;
  const std::vector<int>& off = h->nall > 0 ? h->h_aoff : h->h_poff;
  if (nprob) *nprob = np;
  if (offsets)
    for (int p = 0; p <= np && np > 0; ++p) offsets[p] = off[p];
  return MVAMG_OK;
}

mvamg_status mvamg_batch_small_path(const mvamg_hier* h, int* flags) {
  if (!h || !flags) {
    g_err = "null argument";
    return MVAMG_ERR_ARG;
  }
  const int np = h->nall > 0 ? h->nall : h->nprob;
  for (int p = 0; p < np; ++p) flags[p] = 0;
  for (int p : h->mid) flags[p] = 1;
  return MVAMG_OK;
}

void mvamg_free(mvamg_hier* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  delete h;
}

mvamg_status mvamg_levels(const mvamg_hier* h, int* nlevels, int* n, int64_t* nnz, int* stages) {
  if (!h) {
    g_err = "null handle";
    return MVAMG_ERR_ARG;
  }
  if (nlevels) *nlevels = h->nl;
  for (int l = 0; l < h->nl && l < 32; ++l) {
    if (n) n[l] = h->lev_n[l];
    if (nnz) nnz[l] = h->lev_nnz[l];
    if (stages) stages[l] = (l + 1 < h->nl) ? h->lv[l].ns : 0;
  }
  return MVAMG_OK;
}

mvamg_status mvamg_transfers(const mvamg_hier* h, int* nagg, int64_t* nu) {
  if (!h) {
    g_err = "null handle";
    return MVAMG_ERR_ARG;
  }
  for (int l = 0; l + 1 < h->nl && l < 32; ++l) {
    if (nagg) nagg[l] = h->tr[l].nagg;
    if (nu) nu[l] = h->tr[l].nu;
  }
  return MVAMG_OK;
}

mvamg_status mvamg_set_fine_values(mvamg_hier* h, const double* val, void* stream) {
  try {
    if (!h || !val) throw Error(MVAMG_ERR_ARG, "null argument");
    no_small_path(h);
    check_device(h);
    hipStream_t st = (hipStream_t)stream;
    refill_fine(h, val, st);
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_spmv(mvamg_hier* h, const double* x, double* y, void* stream) {
  try {
    if (!h || !x || !y) throw Error(MVAMG_ERR_ARG, "null argument");
    no_small_path(h);
    check_device(h);
    hipStream_t st = (hipStream_t)stream;
    const int eg = grid_for(h->n);
    k_gather<<<eg, kBlock, 0, st>>>(h->n, h->perm0, x, h->p);
    resid<double, 1>(h, 0, h->lv[0], nullptr, h->p, h->q, M_NONE, st);
    k_scatter<<<eg, kBlock, 0, st>>>(h->n, h->perm0, h->q, y);
    LAUNCHCHECK("spmv");
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_cycle_apply(mvamg_hier* h, const double* r, double* z, int precision, int smoother,
                               void* stream) {
  try {
    if (!h || !r || !z) throw Error(MVAMG_ERR_ARG, "null argument");
    if (r == z) throw Error(MVAMG_ERR_ARG, "r and z must not alias");
    if (precision != 64 && precision != 32) throw Error(MVAMG_ERR_ARG, "precision must be 64 or 32");
    if (smoother != MVAMG_SMOOTH_GS && smoother != MVAMG_SMOOTH_L1JACOBI) throw Error(MVAMG_ERR_ARG, "unknown smoother");
    check_device(h);
    no_small_path(h);
    hipStream_t st = (hipStream_t)stream;
    const int eg = grid_for(h->n);
    k_gather<<<eg, kBlock, 0, st>>>(h->n, h->perm0, r, h->r);
    apply_B(h, h->r, h->z, precision, smoother, st);
    k_scatter<<<eg, kBlock, 0, st>>>(h->n, h->perm0, h->z, z);
    LAUNCHCHECK("cycle_apply");
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_kcycle_apply(mvamg_hier* h, const double* r, double* z, int smoother, void* stream) {
  try {
    if (!h || !r || !z) throw Error(MVAMG_ERR_ARG, "null argument");
    if (r == z) throw Error(MVAMG_ERR_ARG, "r and z must not alias");
    if (smoother != MVAMG_SMOOTH_GS && smoother != MVAMG_SMOOTH_L1JACOBI) throw Error(MVAMG_ERR_ARG, "unknown smoother");
    check_device(h);
    no_small_path(h);
    hipStream_t st = (hipStream_t)stream;
    const int eg = grid_for(h->n);
    k_gather<<<eg, kBlock, 0, st>>>(h->n, h->perm0, r, h->r);
    apply_B(h, h->r, h->z, 64, smoother, st, MVAMG_CYCLE_K);
    k_scatter<<<eg, kBlock, 0, st>>>(h->n, h->perm0, h->z, z);
    LAUNCHCHECK("kcycle_apply");
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_cycle_apply_noalloc(mvamg_hier* h, const double* r, double* z, int precision, int smoother,
                                       void* stream) {
  try {
    if (!h || !r || !z) throw Error(MVAMG_ERR_ARG, "null argument");
    if (r == z) throw Error(MVAMG_ERR_ARG, "r and z must not alias");
    if (precision != 64 && precision != 32) throw Error(MVAMG_ERR_ARG, "precision must be 64 or 32");
    if (smoother != MVAMG_SMOOTH_GS && smoother != MVAMG_SMOOTH_L1JACOBI) throw Error(MVAMG_ERR_ARG, "unknown smoother");
    check_device(h);
    no_small_path(h);
    if (h->prof) throw Error(MVAMG_ERR_ARG, "measurement is on (mvamg_profile): its events are created per launch");
    const size_t need = ScratchWork(h, precision, nullptr).bytes();
    if (need > (size_t)MVAMG_NOALLOC_SCRATCH_BYTES)
      throw Error(MVAMG_ERR_ARG, "cycle work space of " + std::to_string(need) + " bytes exceeds the " +
                                     std::to_string((size_t)MVAMG_NOALLOC_SCRATCH_BYTES) + "-byte static scratch");
    unsigned char* base = scratch_address(h->device);
    hipStream_t st = (hipStream_t)stream;
    const int eg = grid_for(h->n);
    ScratchWork work(h, precision, base);
    k_gather<<<eg, kBlock, 0, st>>>(h->n, h->perm0, r, h->r);
    apply_B(h, h->r, h->z, precision, smoother, st);
    k_scatter<<<eg, kBlock, 0, st>>>(h->n, h->perm0, h->z, z);
    LAUNCHCHECK("cycle_apply_noalloc");
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_pcg_solve(mvamg_hier* h, const int* rowptr, const int* col, const double* val, const double* b,
                             double* x, const mvamg_solve_params* prm, mvamg_info* info, void* stream) {
  try {
    if (!h) throw Error(MVAMG_ERR_ARG, "null handle");
    if (!prm || !b || !x) throw Error(MVAMG_ERR_ARG, "null argument");
    if (h->nprob > 0 || h->nall > 0) throw Error(MVAMG_ERR_ARG, "a batch handle is solved with mvamg_batch_pcg_solve");
    check_device(h);
    use_matrix(h, rowptr, col, val, (hipStream_t)stream);
    return pcg(h, b, x, prm, info, (hipStream_t)stream);
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_adjoint_solve(mvamg_hier* h, const int* rowptr, const int* col, const double* val,
                                 const double* dLdx, double* lambda, const mvamg_solve_params* prm, mvamg_info* info,
                                 void* stream) {
  try {
    if (!h || !lambda || !prm || !dLdx) throw Error(MVAMG_ERR_ARG, "null argument");
    if (h->nprob > 0 || h->nall > 0) throw Error(MVAMG_ERR_ARG, "a batch handle is solved with mvamg_batch_pcg_solve");
    check_device(h);
    hipStream_t st = (hipStream_t)stream;
    use_matrix(h, rowptr, col, val, st);
    HIPCHECK(hipMemsetAsync(lambda, 0, sizeof(double) * (size_t)h->n, st));
    return pcg(h, dLdx, lambda, prm, info, st);
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_grad_coeffs(mvamg_hier* h, const double* lambda, const double* x, double* dval, void* stream) {
  try {
    if (!h || !lambda || !x || !dval) throw Error(MVAMG_ERR_ARG, "null argument");
    check_device(h);
    no_small_path(h);
    hipStream_t st = (hipStream_t)stream;
    k_grad_coeffs<<<grid_for(h->n), kBlock, 0, st>>>(h->n, h->frp, h->fci, lambda, x, dval);
    LAUNCHCHECK("grad_coeffs");
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_spmv_block(mvamg_hier* h, const double* X, double* Y, int m, void* stream) {
  try {
    if (!h || !X || !Y) throw Error(MVAMG_ERR_ARG, "null argument");
    if (m < 1 || m > MVAMG_BLOCK_MAX) throw Error(MVAMG_ERR_ARG, "block width must be 1..32");
    check_device(h);
    hipStream_t st = (hipStream_t)stream;
    ensure_block(h);
    k_bgather<<<bgrid_elem(h->n), kBlock, 0, st>>>(h->n, h->perm0, m, X, h->bp);
    bresid<double, 2>(h, h->lv[0], nullptr, h->bp, h->bq, MM_STORE_R0, st);
    k_bscatter<<<bgrid_elem(h->n), kBlock, 0, st>>>(h->n, h->perm0, m, h->bq, Y);
    LAUNCHCHECK("spmv_block");
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_cycle_apply_block(mvamg_hier* h, const double* R, double* Z, int m, int precision, int smoother,
                                     void* stream) {
  try {
    if (!h || !R || !Z) throw Error(MVAMG_ERR_ARG, "null argument");
    if (R == Z) throw Error(MVAMG_ERR_ARG, "R and Z must not alias");
    if (m < 1 || m > MVAMG_BLOCK_MAX) throw Error(MVAMG_ERR_ARG, "block width must be 1..32");
    if (precision != 64 && precision != 32) throw Error(MVAMG_ERR_ARG, "precision must be 64 or 32");
    if (smoother != MVAMG_SMOOTH_GS && smoother != MVAMG_SMOOTH_L1JACOBI) throw Error(MVAMG_ERR_ARG, "unknown smoother");
    check_device(h);
    hipStream_t st = (hipStream_t)stream;
    ensure_block(h);
    DevLevel& L0 = h->lv[0];
    k_bgather<<<bgrid_elem(h->n), kBlock, 0, st>>>(h->n, h->perm0, m, R, L0.br);
    bapply_B(h, L0.br, L0.bx, precision, smoother, st);
    k_bscatter<<<bgrid_elem(h->n), kBlock, 0, st>>>(h->n, h->perm0, m, L0.bx, Z);
    LAUNCHCHECK("cycle_apply_block");
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_pcg_solve_block(mvamg_hier* h, const double* B, double* X, int m, const mvamg_solve_params* prm,
                                   mvamg_info* info, void* stream) {
  try {
    if (!h) throw Error(MVAMG_ERR_ARG, "null handle");
    if (m < 1 || m > MVAMG_BLOCK_MAX) throw Error(MVAMG_ERR_ARG, "block width must be 1..32");
    if (prm && prm->cycle != MVAMG_CYCLE_V) throw Error(MVAMG_ERR_ARG, "block solves run the V-cycle only");
    check_device(h);
    ensure_block(h);
    BlockOps O(h, m);
    return multi_pcg(O, B, X, prm, info, (hipStream_t)stream);
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_batch_pcg_solve(mvamg_hier* h, const double* b, double* x, const mvamg_solve_params* prm,
                                   mvamg_info* info, void* stream) {
  try {
    if (!h) throw Error(MVAMG_ERR_ARG, "null handle");
    if (h->nprob < 1 && h->nall < 1) throw Error(MVAMG_ERR_ARG, "not a batch handle (use mvamg_pcg_solve)");
    if (prm && prm->cycle != MVAMG_CYCLE_V) throw Error(MVAMG_ERR_ARG, "batch solves run the V-cycle only");
    check_device(h);
    hipStream_t st = (hipStream_t)stream;
    if (h->nmini == 0) {
      BatchOps O(h);
      return multi_pcg(O, b, x, prm, info, st);
    }
    // problems on the small path: one launch on the second stream, the
    // lockstep part meanwhile on st; results in the caller's problem order
    if (!prm || !b || !x) throw Error(MVAMG_ERR_ARG, "null argument");
    if (prm->precision != 64) throw Error(MVAMG_ERR_ARG, "the small-problem path runs the binary64 cycle only");
    if (prm->smoother != MVAMG_SMOOTH_GS && prm->smoother != MVAMG_SMOOTH_L1JACOBI)
      throw Error(MVAMG_ERR_ARG, "unknown smoother");
    if (prm->maxit < 0 || !(prm->rtol >= 0.0)) throw Error(MVAMG_ERR_ARG, "invalid maxit or rtol");
    mini_launch(h, b, x, prm, st);
    mvamg_status su = MVAMG_OK;
    try {
      if (h->nprob > 0) {
        const int nu = h->nprob;
        std::vector<mvamg_info> ui(nu);
        std::vector<double> uh;
        mvamg_solve_params up = *prm;
        if (prm->history) {
          uh.assign((size_t)nu * (prm->maxit + 1), 0.0);
          up.history = uh.data();
        }
        BatchOps O(h);
        su = multi_pcg(O, b, x, &up, ui.data(), st);
        for (int q = 0; q < nu; ++q) {
          const int p = h->uid[q];
          if (info) info[p] = ui[q];
          if (prm->history)
            std::memcpy(prm->history + (size_t)p * (prm->maxit + 1), uh.data() + (size_t)q * (prm->maxit + 1),
                        sizeof(double) * (prm->maxit + 1));
        }
      }
    } catch (...) {
      (void)hipStreamSynchronize(h->mstream);
      throw;
    }
    const bool mall = mini_collect(h, prm, info, st);
    return (su == MVAMG_OK && mall) ? MVAMG_OK : MVAMG_NOT_CONVERGED;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_setup_bases(int n_level, int m, int nagg, int max_na, const int* aptr, const int* arows,
                               const double* W, double tol, int* k, double* U, double* dropped, int* flag,
                               void* stream) {
  try {
    if (!aptr || !arows || !W || !k || !U || !dropped || !flag) throw Error(MVAMG_ERR_ARG, "null argument");
    setup_bases(m, nagg, max_na, aptr, arows, W, tol, n_level, k, U, dropped, flag, (hipStream_t)stream);
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_setup_pattern(int n, const int* rowptr, const int* col, int nagg, const int* aptr,
                                 const int* arows, const int* k, int* agg, int* loc, int* coff, int* cagg,
                                 int* crp, int* ccol, int64_t* nnz) {
  try {
    if (!rowptr || !col || !aptr || !arows || !k || !agg || !loc || !coff || !cagg || !nnz)
      throw Error(MVAMG_ERR_ARG, "null argument");
    if ((crp == nullptr) != (ccol == nullptr)) throw Error(MVAMG_ERR_ARG, "crp and ccol are passed together");
    *nnz = galerkin_pattern(n, rowptr, col, nagg, aptr, arows, k, agg, loc, coff, cagg, crp, ccol);
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_setup_galerkin(int m, int nagg, int nc, const int* aptr, const int* arows, const int* coff,
                                  const int* agg, const int* loc, const int* cagg, const int* rowptr, const int* col,
                                  const double* val, const double* U, const int* crp, const int* ccol,
                                  double* cval, double* work, int* flag, void* stream) {
  try {
    if (!aptr || !arows || !coff || !agg || !loc || !cagg || !rowptr || !col || !val || !U || !crp || !ccol ||
        !cval || !work || !flag)
      throw Error(MVAMG_ERR_ARG, "null argument");
    if (m < 1 || m > kSvdMaxM || nagg < 1 || nc < 1) throw Error(MVAMG_ERR_ARG, "sizes out of range");
    hipStream_t st = (hipStream_t)stream;
    k_fill<int><<<1, kBlock, 0, st>>>(1, 0, flag);
    // few aggregates (a coarse level): several waves per aggregate, or the
    // device would hold a handful of long waves
    if (nagg < kGalSplitBelow)
      k_setup_galerkin_split<<<nagg, 64 * kGalWaves, 0, st>>>(m, nagg, aptr, arows, coff, agg, loc, cagg, rowptr,
                                                              col, val, U, crp, ccol, work);
    else
      k_setup_galerkin<<<nagg, 64, 0, st>>>(m, nagg, aptr, arows, coff, agg, loc, cagg, rowptr, col, val, U, crp,
                                            ccol, work);
    k_symmetrize<<<grid_for(nc), kBlock, 0, st>>>(nc, crp, ccol, work, cval, flag);
    LAUNCHCHECK("setup_galerkin");
    int hflag = 0;
    HIPCHECK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    if (hflag) throw Error(MVAMG_ERR_ARG, "coarse pattern is not symmetric (A's pattern must be)");
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_setup_restrict(int m, int nagg, const int* aptr, const int* arows, const int* coff,
                                  const double* U, const double* W, double* Wc, void* stream) {
  try {
    if (!aptr || !arows || !coff || !U || !W || !Wc) throw Error(MVAMG_ERR_ARG, "null argument");
    if (m < 1 || m > kSvdMaxM || nagg < 1) throw Error(MVAMG_ERR_ARG, "sizes out of range");
    k_setup_restrict<<<nagg, 64, 0, (hipStream_t)stream>>>(m, nagg, aptr, arows, coff, U, W, Wc);
    LAUNCHCHECK("setup_restrict");
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_composite_work_bytes(int n, size_t* bytes) {
  if (n < 1 || !bytes) {
    g_err = "n must be positive and bytes not null";
    return MVAMG_ERR_ARG;
  }
  *bytes = composite_work_bytes(n);
  return MVAMG_OK;
}

namespace {
void check_comp_args(int cycle, int smoother) {
  if (cycle != MVAMG_CYCLE_V && cycle != MVAMG_CYCLE_K) throw Error(MVAMG_ERR_ARG, "unknown cycle");
  if (smoother != MVAMG_SMOOTH_GS && smoother != MVAMG_SMOOTH_L1JACOBI) throw Error(MVAMG_ERR_ARG, "unknown smoother");
}
}  // namespace

mvamg_status mvamg_composite_apply(mvamg_hier* const* hs, int r, int cycle, int smoother, const double* res,
                                   double* z, void* work, size_t work_bytes, void* stream) {
  try {
    if (!res || !z || res == z) throw Error(MVAMG_ERR_ARG, "null or aliased vectors");
    check_comp_args(cycle, smoother);
    hipStream_t st = (hipStream_t)stream;
    check_composite(hs, r, st);
    const CompWork w = comp_work(hs[0]->n, work, work_bytes);
    comp_apply(hs, r, cycle, smoother, res, z, w, st);
    LAUNCHCHECK("composite_apply");
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_composite_test(mvamg_hier* const* hs, int r, int cycle, int smoother, int nu, double* x,
                                  double* rho, void* work, size_t work_bytes, void* stream) {
  try {
    if (!x || !rho || nu < 1) throw Error(MVAMG_ERR_ARG, "null argument or nu < 1");
    check_comp_args(cycle, smoother);
    hipStream_t st = (hipStream_t)stream;
    check_composite(hs, r, st);
    const CompWork w = comp_work(hs[0]->n, work, work_bytes);
    *rho = comp_test(hs, r, cycle, smoother, nu, x, w, st);
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_composite_pcg_solve(mvamg_hier* const* hs, int r, const double* b, double* x,
                                       const mvamg_solve_params* prm, mvamg_info* info, void* work,
                                       size_t work_bytes, void* stream) {
  try {
    if (!prm || !b || !x) throw Error(MVAMG_ERR_ARG, "null argument");
    if (prm->precision != 64) throw Error(MVAMG_ERR_ARG, "the composite runs in binary64 only");
    if (prm->maxit < 0 || !(prm->rtol >= 0.0)) throw Error(MVAMG_ERR_ARG, "invalid maxit or rtol");
    check_comp_args(prm->cycle, prm->smoother);
    hipStream_t st = (hipStream_t)stream;
    check_composite(hs, r, st);
    const CompWork w = comp_work(hs[0]->n, work, work_bytes);
    return comp_pcg(hs, r, b, x, prm, info, w, st);
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_autotune(mvamg_hier* h, int what, char* report, size_t cap, void* stream) {
  try {
    if (!h) throw Error(MVAMG_ERR_ARG, "null handle");
    if (what & ~MVAMG_TUNE_ALL) throw Error(MVAMG_ERR_ARG, "unknown tuning bits");
    check_device(h);
    hipStream_t st = (hipStream_t)stream;
    const bool prof = h->prof;
    h->prof = false;
    std::string rep;
    try {
      if (what & MVAMG_TUNE_GROUP_LANES) tune_group_lanes(h, st, rep);
      if ((what & MVAMG_TUNE_BLOCK_COARSE) && h->nprob == 0 && h->nall == 0) {
        if (block_fits(h))
          tune_block_coarse(h, st, rep);
        else
          rep += "gemm: skipped (the arena has no block work space); ";
      }
      if (what & MVAMG_TUNE_BATCH_CHUNKS) tune_batch_chunks(h, st, rep);
    } catch (...) {
      h->prof = prof;
      throw;
    }
    h->prof = prof;
    HIPCHECK(hipStreamSynchronize(st));
    drop_graphs(h);
    rep += "chosen: " + tune_text(h);
    if (report && cap > 0) {
      const size_t k = std::min(cap - 1, rep.size());
      std::memcpy(report, rep.data(), k);
      report[k] = 0;
    }
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_tune_get(const mvamg_hier* h, char* buf, size_t cap) {
  try {
    if (!h) throw Error(MVAMG_ERR_ARG, "null handle");
    copy_text(tune_text(h), buf, cap);
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_tune_set(mvamg_hier* h, const char* text) {
  try {
    if (!h || !text) throw Error(MVAMG_ERR_ARG, "null argument");
    check_device(h);
    HIPCHECK(hipDeviceSynchronize());
    apply_tune_text(h, text);
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

mvamg_status mvamg_signature(const mvamg_hier* h, char* buf, size_t cap) {
  try {
    if (!h) throw Error(MVAMG_ERR_ARG, "null handle");
    copy_text(signature_text(h), buf, cap);
    return MVAMG_OK;
  } catch (const Error& e) {
    return fail_status(e);
  }
}

}  // extern "C"
