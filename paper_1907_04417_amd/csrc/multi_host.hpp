// Host driver for several systems at once (included by mvamg_lib.hip inside
// its internal namespace, after the single-system helpers):
//   * block right-hand sides: up to 32 columns through one hierarchy, every
//     level operator applied to n x 32 row-major blocks;
//   * a batch: independent problems uploaded as one block-diagonal
//     hierarchy (level l of the batch = level l of every problem, stage c =
//     stage c of every problem), so one launch covers one step of all of them.
// Each system (column or problem) keeps its own conjugate-gradient scalars
// and stops on its own residual; the host loop is shared.

template <typename T>
T* pick(double* d, float* f) {
  if constexpr (std::is_same<T, double>::value)
    return d;
  else
    return f;
}

// Variants of the coarsest block product Z = A_L^{-1} R (chosen by the
// autotuner): vector FMA with one row per half wave, or MFMA with W waves per
// 16-row tile and the inner dimension split KS ways.
struct GemmVariant {
  int mfma, W, KS;
};
constexpr GemmVariant kGemmVariants[] = {{0, 0, 1}, {1, 16, 1}, {1, 4, 2}, {1, 4, 4}, {1, 4, 8}, {1, 2, 8}};
constexpr int kGemmVariantCount = sizeof(kGemmVariants) / sizeof(kGemmVariants[0]);
constexpr int kGemmDefault = 4;
constexpr int kGemmMaxSplit = 8;
// most partial-sum chunks per problem of the batch reductions (autotuned)
constexpr int kMaxChunks = 64;

// ----------------------------------------------------- work arrays

void ensure_multi(mvamg_hier* h, int nsys, int nparts) {
  MultiBufs& M = h->mb;
  if (M.nsys >= nsys && M.nparts >= nparts) return;
  M.nsys = std::max(M.nsys, nsys);
  M.nparts = std::max(M.nparts, nparts);
  if (M.scal) h->dfree(M.scal);
  if (M.part) h->dfree(M.part);
  if (M.act) h->dfree(M.act);
  if (M.pinned) (void)hipHostFree(M.pinned);
  if (M.pact) (void)hipHostFree(M.pact);
  M.pinned = M.pact = nullptr;
  M.scal = h->dalloc<double>((size_t)M.nsys * S_NSCAL);
  M.part = h->dalloc<double>(2 * (size_t)M.nsys * M.nparts);
  M.act = h->dalloc<double>(M.nsys);
  if (h->sizing()) return;
  HIPCHECK(hipHostMalloc((void**)&M.pinned, (size_t)M.nsys * S_NSCAL * sizeof(double), hipHostMallocDefault));
  HIPCHECK(hipHostMalloc((void**)&M.pact, (size_t)M.nsys * sizeof(double), hipHostMallocDefault));
  // graphs captured earlier hold the old addresses
  for (auto it = h->graphs.begin(); it != h->graphs.end();) {
    if (it->first >= 1000) {
      (void)hipGraphExecDestroy(it->second);
      it = h->graphs.erase(it);
    } else {
      ++it;
    }
  }
}

// grid of a row-per-half-wave kernel whose column partials are reduced afterwards
int bgrid_for(int64_t rows) {
  int64_t b = (rows + kRowsPerBlock - 1) / kRowsPerBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 2048));
}
int bgrid_elem(int64_t rows) {
  int64_t b = (rows + kRowsPerBlock - 1) / kRowsPerBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 65535));
}

// grid of the block residual kernels (grid-stride).  With per-column
// partial sums (MODE 1) at most one block per slab (or per four groups),
// capped at kMaxBlockParts partials per column; otherwise one row per half
// wave (one group per wave).
constexpr int kMaxBlockParts = 16384;
int bresid_grid(const DevLevel& L, int mode) {
  if (L.sell) {
    const int64_t b = (mode == 1) ? L.nslabs : (int64_t)L.nslabs * (64 / kRowsPerBlock);
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, mode == 1 ? kMaxBlockParts : (int64_t)1 << 24));
  }
  const int64_t b = (L.ng + 3) / 4;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, mode == 1 ? kMaxBlockParts : (int64_t)1 << 24));
}

int block_nparts(const mvamg_hier* h) {
  int nparts = 2048;
  for (int l = 0; l + 1 < h->nl; ++l) nparts = std::max(nparts, bresid_grid(h->lv[l], 1));
  return nparts;
}

// Bytes of every array ensure_block takes, in the order it takes them.
std::vector<size_t> block_request(const mvamg_hier* h) {
  std::vector<size_t> b;
  for (int l = 0; l < h->nl; ++l) {
    const size_t m = (size_t)h->lv[l].n * kNB;
    b.insert(b.end(), {8 * m, 8 * m, 4 * m, 4 * m});
    if (l + 1 < h->nl) b.insert(b.end(), {8 * m, 4 * m});
  }
  const size_t m0 = (size_t)h->n * kNB;
  b.insert(b.end(), {8 * m0, 8 * m0, 8 * m0, 8 * m0});
  b.insert(b.end(), {8 * (size_t)h->co.n * kNB, 8 * (size_t)h->co.n * kNB, 8 * (size_t)kGemmMaxSplit * h->co.n * kNB});
  const MultiBufs& M = h->mb;
  if (M.nsys < kNB || M.nparts < block_nparts(h)) {
    const size_t nsys = std::max(M.nsys, kNB), np = std::max(M.nparts, block_nparts(h));
    b.insert(b.end(), {8 * nsys * S_NSCAL, 16 * nsys * np, 8 * nsys});
  }
  return b;
}

// Whether the arena still has room for the block work space.
bool block_fits(const mvamg_hier* h) { return h->blk_ready || h->fits(block_request(h)); }

void ensure_block(mvamg_hier* h) {
  if (h->blk_ready) return;
  if (h->nprob > 0 || h->nall > 0)
    throw Error(MVAMG_ERR_ARG, "block right-hand sides are not supported on a batch of problems");
  for (int l = 0; l < h->nl; ++l)
    if ((int64_t)h->lev_n[l] * kNB >= ((int64_t)1 << 31)) throw Error(MVAMG_ERR_ARG, "level too large for 32-column blocks");
  if (!block_fits(h))
    throw Error(MVAMG_ERR_ARG, "the arena has no room for the block work space (size it with nrhs > 1)");
  for (int l = 0; l < h->nl; ++l) {
    DevLevel& L = h->lv[l];
    const size_t m = (size_t)L.n * kNB;
    L.br = h->dalloc<double>(m);
    L.bx = h->dalloc<double>(m);
    L.br32 = h->dalloc<float>(m);
    L.bx32 = h->dalloc<float>(m);
    if (l + 1 < h->nl) {
      L.bs = h->dalloc<double>(m);
      L.bs32 = h->dalloc<float>(m);
    }
  }
  const size_t m0 = (size_t)h->n * kNB;
  h->bb = h->dalloc<double>(m0);
  h->bxv = h->dalloc<double>(m0);
  h->bp = h->dalloc<double>(m0);
  h->bq = h->dalloc<double>(m0);
  h->co.br = h->dalloc<double>((size_t)h->co.n * kNB);
  h->co.bz = h->dalloc<double>((size_t)h->co.n * kNB);
  h->co.bsplit = h->dalloc<double>((size_t)kGemmMaxSplit * h->co.n * kNB);
  ensure_multi(h, kNB, block_nparts(h));
  h->blk_ready = true;
}

// --------------------------------------------- block-vector level operators

template <typename T>
double bstage_bytes(const DevLevel& L, int c) {
  return (double)L.stage_nnz[c] * (sizeof(T) + 4) + (double)L.stage_rows[c] * (4 + 3.0 * kNB * sizeof(T));
}

template <typename T>
void bgs_stage(mvamg_hier* h, int l, const DevLevel& L, int c, const T* r, T* x, int backward, hipStream_t st,
               bool first_sweep = false) {
  const int kc = (l == 0) ? MVAMG_KC_SMOOTH_FINE : MVAMG_KC_SMOOTH_COARSE;
  const double by = bstage_bytes<T>(L, c);
  if (L.sell) {
    const int s0 = L.h_sslab[c], s1 = L.h_sslab[c + 1];
    if (s1 <= s0) return;
    const int grid = (s1 - s0) * (64 / kRowsPerBlock);
    klaunch(h, kc, by, k_bgs_sell<T>, grid, kBlock, st, L.slabs, s0, s1, L.col, lval<T>(L), ldblk<T>(L), r, x,
            first_sweep ? L.h_srow[c] : INT_MAX);
  } else {
    const int g0 = L.h_sgrp[c], g1 = L.h_sgrp[c + 1];
    if (g1 <= g0) return;
    if (L.gshared) {  // block per group over the shared column lists
      switch (L.G0) {
        case 1: klaunch(h, kc, by, k_bgs_grps<T, 1>, g1 - g0, kBlock, st, g0, g1, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, backward); break;
        case 2: klaunch(h, kc, by, k_bgs_grps<T, 2>, g1 - g0, kBlock, st, g0, g1, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, backward); break;
        case 4: klaunch(h, kc, by, k_bgs_grps<T, 4>, g1 - g0, kBlock, st, g0, g1, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, backward); break;
        default: klaunch(h, kc, by, k_bgs_grps<T, 8>, g1 - g0, kBlock, st, g0, g1, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, backward); break;
      }
      LAUNCHCHECK("bgs_stage");
      return;
    }
    const int grid = (g1 - g0 + 3) / 4;
    switch (L.G) {
      case 1: klaunch(h, kc, by, k_bgs_grp<T, 1>, grid, kBlock, st, g0, g1, L.rec, L.col, lval<T>(L), ldblk<T>(L), r, x, backward); break;
      case 2: klaunch(h, kc, by, k_bgs_grp<T, 2>, grid, kBlock, st, g0, g1, L.rec, L.col, lval<T>(L), ldblk<T>(L), r, x, backward); break;
      case 4: klaunch(h, kc, by, k_bgs_grp<T, 4>, grid, kBlock, st, g0, g1, L.rec, L.col, lval<T>(L), ldblk<T>(L), r, x, backward); break;
      default: klaunch(h, kc, by, k_bgs_grp<T, 8>, grid, kBlock, st, g0, g1, L.rec, L.col, lval<T>(L), ldblk<T>(L), r, x, backward); break;
    }
  }
  LAUNCHCHECK("bgs_stage");
}

template <typename T>
void bzero_stage0(mvamg_hier* h, int l, const DevLevel& L, const T* r, T* x, hipStream_t st) {
  const int kc = (l == 0) ? MVAMG_KC_SMOOTH_FINE : MVAMG_KC_SMOOTH_COARSE;
  const double by = ((double)L.n + 2.0 * L.stage_rows[0]) * kNB * sizeof(T);
  if (L.sell) {
    klaunch(h, kc, 3.0 * L.rows0 * kNB * sizeof(T), k_bstage0_point<T>, bgrid_elem(L.rows0), kBlock, st, L.rows0,
            ldblk<T>(L), r, x);
  } else {
    klaunch(h, kc, by, k_bzero_stage0_grp<T>, bgrid_elem(L.ng), kBlock, st, L.ng, L.h_sgrp[1], L.gstart, L.dboff, ldblk<T>(L), r, x);
  }
  LAUNCHCHECK("bzero_stage0");
}

// MODE 0: s = r - A x; MODE 1: s = A x and per-column x.s reduced by `mode`; MODE 2: s = A x
// nst >= 0 (MODE 0): only the rows of stages [0, nst), as resid.
template <typename T, int MODE>
void bresid(mvamg_hier* h, const DevLevel& L, const T* r, const T* x, T* s, int mode, hipStream_t st, int nst = -1) {
  const int kc = MODE != 0 ? MVAMG_KC_SPMV : MVAMG_KC_RESIDUAL;
  const bool part_rows = MODE == 0 && nst >= 0 && nst < L.ns;
  const double by = part_rows ? resid_stage_bytes<T>(h, L, nst, 3.0 * kNB * sizeof(T), false)
                              : (double)L.nnz * (sizeof(T) + 4) + 4.0 * (L.n + 1) +
                                    (double)L.n * kNB * sizeof(T) * (MODE != 0 ? 2 : 3);
  int grid = bresid_grid(L, MODE);
  double* part = h->mb.part;
  if (L.sell) {
    const int ns = part_rows ? L.h_sslab[nst] : L.nslabs;
    if (part_rows) grid = std::max(1, std::min(grid, ns * (64 / kRowsPerBlock)));
    // slabs in spatial order where the rows span several stages (their
    // neighbours' rows are then read by one XCD, close in time)
    const Slab* sl = !part_rows ? L.bslab_full : (nst == L.ns - 1 ? L.bslab_part : L.slabs);
    if (ns > 0)
      klaunch(h, kc, by, k_bresid_sell<T, MODE>, grid, kBlock, st, sl, ns, L.col, lval<T>(L), ldblk<T>(L), r, x, s, part);
  } else {
    const int ng = part_rows ? L.h_sgrp[nst] : L.ng;
    if (part_rows) grid = std::max(1, std::min(grid, (ng + 3) / 4));
    if (MODE == 0 && L.gshared && ng > 0) {  // block per group over the shared column lists
      switch (L.G0) {
        case 1: klaunch(h, kc, by, k_bresid_grps<T, 1>, ng, kBlock, st, ng, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, s); break;
        case 2: klaunch(h, kc, by, k_bresid_grps<T, 2>, ng, kBlock, st, ng, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, s); break;
        case 4: klaunch(h, kc, by, k_bresid_grps<T, 4>, ng, kBlock, st, ng, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, s); break;
        default: klaunch(h, kc, by, k_bresid_grps<T, 8>, ng, kBlock, st, ng, L.rec, L.gcol, lval<T>(L), ldblk<T>(L), r, x, s); break;
      }
    } else if (ng > 0) switch (L.G) {
      case 1: klaunch(h, kc, by, k_bresid_grp<T, 1, MODE>, grid, kBlock, st, ng, L.rec, L.col, lval<T>(L), ldblk<T>(L), r, x, s, part); break;
      case 2: klaunch(h, kc, by, k_bresid_grp<T, 2, MODE>, grid, kBlock, st, ng, L.rec, L.col, lval<T>(L), ldblk<T>(L), r, x, s, part); break;
      case 4: klaunch(h, kc, by, k_bresid_grp<T, 4, MODE>, grid, kBlock, st, ng, L.rec, L.col, lval<T>(L), ldblk<T>(L), r, x, s, part); break;
      default: klaunch(h, kc, by, k_bresid_grp<T, 8, MODE>, grid, kBlock, st, ng, L.rec, L.col, lval<T>(L), ldblk<T>(L), r, x, s, part); break;
    }
  }
  LAUNCHCHECK("bresid");
  if (MODE == 1) {
    k_mfinish<1><<<kNB, kBlock, 0, st>>>(kNB, grid, part, h->mb.scal, mode);
    LAUNCHCHECK("bresid finish");
  }
}

void launch_bgemm(mvamg_hier* h, int variant, const double* R, double* Z, hipStream_t st) {
  DevCoarse& C = h->co;
  const double by = 8.0 * C.n * (double)C.n + 2.0 * C.n * kNB * 8.0;
  const GemmVariant v = kGemmVariants[variant < 0 ? kGemmDefault : variant];
  const int nt = (C.n + 15) / 16;
  double* out = (v.KS == 1) ? Z : C.bsplit;
  if (!v.mfma) {
    klaunch(h, MVAMG_KC_COARSE, by, k_bgemm<1>, C.np / 8, kBlock, st, C.n, C.np, C.Ainv, R, Z);
  } else {
    const dim3 grid(nt, v.KS);
    switch (v.W) {
      case 16: klaunch(h, MVAMG_KC_COARSE, by, k_bgemm_mfma<16>, grid, dim3(1024), st, C.n, C.np, C.Ainv, R, out); break;
      case 8: klaunch(h, MVAMG_KC_COARSE, by, k_bgemm_mfma<8>, grid, dim3(512), st, C.n, C.np, C.Ainv, R, out); break;
      case 4: klaunch(h, MVAMG_KC_COARSE, by, k_bgemm_mfma<4>, grid, dim3(256), st, C.n, C.np, C.Ainv, R, out); break;
      default: klaunch(h, MVAMG_KC_COARSE, by, k_bgemm_mfma<2>, grid, dim3(128), st, C.n, C.np, C.Ainv, R, out); break;
    }
    if (v.KS > 1) {
      const int m = C.n * kNB;
      k_bsum_splits<<<grid_elem(m), kBlock, 0, st>>>(m, v.KS, C.bsplit, Z);
    }
  }
  LAUNCHCHECK("bgemm");
}

template <typename T>
void bcoarse_solve(mvamg_hier* h, const T* r, T* z, hipStream_t st) {
  DevCoarse& C = h->co;
  if constexpr (std::is_same<T, double>::value) {
    launch_bgemm(h, h->gemm_variant, r, z, st);
  } else {
    k_cast<float, double><<<grid_elem((int64_t)C.n * kNB), kBlock, 0, st>>>(C.n * kNB, r, C.br);
    launch_bgemm(h, h->gemm_variant, C.br, C.bz, st);
    k_cast<double, float><<<grid_elem((int64_t)C.n * kNB), kBlock, 0, st>>>(C.n * kNB, C.bz, z);
  }
  LAUNCHCHECK("bcoarse_solve");
}

// X = B_l R for block vectors (one V-cycle from a zero guess per column)
template <typename T>
void bvcycle(mvamg_hier* h, int l, const T* r, T* x, int smoother, hipStream_t st, bool x_started = false,
             bool stage0_written = false) {
  if (l == h->nl - 1) {
    bcoarse_solve<T>(h, r, x, st);
    return;
  }
  DevLevel& L = h->lv[l];
  DevLevel& C = h->lv[l + 1];
  const DevTransfer& P = h->tr[l];
  T* s = pick<T>(L.bs, L.bs32);
  T* rc = pick<T>(C.br, C.br32);
  T* xc = pick<T>(C.bx, C.bx32);
  if (smoother == MVAMG_SMOOTH_GS) {
    // stage0_written: a point level's stage 0 of the sweep from zero is
    // already in x (written with r by the CG update); the other rows are not set
    if (!x_started && !stage0_written) bzero_stage0<T>(h, l, L, r, x, st);
    for (int c = 1; c < L.ns; ++c) bgs_stage<T>(h, l, L, c, r, x, 0, st, !x_started && L.sell);
  } else if (!x_started) {
    k_bl1_init<T><<<bgrid_elem(L.n), kBlock, 0, st>>>(L.n, ldl1<T>(L), r, x);
  }
  // rows of a point level's last stage have zero residual after the sweep (as in vcycle)
  const bool zero_last = smoother == MVAMG_SMOOTH_GS && L.ng == L.n;
  bresid<T, 0>(h, L, r, x, s, MM_STORE_R0, st, zero_last ? L.ns - 1 : -1);
  const int scut = zero_last ? L.h_srow[L.ns - 1] : L.n;
  const int tg = (P.nagg + 3) / 4;
  const double tby = (double)P.nu * sizeof(T) + 4.0 * L.n + (double)scut * kNB * sizeof(T) + (double)C.n * kNB * sizeof(T);
  const bool next_smoothed = (l + 2 < h->nl);
  // KMAX: the transfer's widest aggregate basis rounded up to 1, 2, 4 or 8
  auto launch = [&](auto km, auto init) {
    constexpr int KM = decltype(km)::value, IN = decltype(init)::value;
    const double by = tby + (IN == 0 ? 0.0 : (double)C.n * kNB * sizeof(T));
    klaunch(h, MVAMG_KC_RESTRICT, by, k_brestrict<T, KM, IN>, tg, kBlock, st, P.nagg, P.arec, P.arows, tU<T>(P), s,
            scut, rc, IN == 1 ? ldblk<T>(C) : (const T*)nullptr, IN == 2 ? ldl1<T>(C) : (const T*)nullptr,
            IN == 0 ? (T*)nullptr : xc);
  };
  auto by_init = [&](auto km) {
    if (!next_smoothed)
      launch(km, std::integral_constant<int, 0>{});
    else if (smoother == MVAMG_SMOOTH_GS)
      launch(km, std::integral_constant<int, 1>{});
    else
      launch(km, std::integral_constant<int, 2>{});
  };
  switch (P.kmax) {
    case 1: by_init(std::integral_constant<int, 1>{}); break;
    case 2: by_init(std::integral_constant<int, 2>{}); break;
    case 3:
    case 4: by_init(std::integral_constant<int, 4>{}); break;
    default: by_init(std::integral_constant<int, 8>{}); break;
  }
  LAUNCHCHECK("brestrict");
  bvcycle<T>(h, l + 1, rc, xc, smoother, st, next_smoothed);
  {
    // rows overwritten unread by the backward sweep's first stage are skipped
    const bool gs = smoother == MVAMG_SMOOTH_GS;
    const int nr = gs ? P.ncut : P.nf;
    const double nu = gs ? (double)P.nu_cut : (double)P.nu;
    const int pg = bgrid_elem(std::max(nr, 1));
    const double pby = nu * sizeof(T) + (double)nr * (4 + 2.0 * kNB * sizeof(T)) + (double)C.n * kNB * sizeof(T);
    if (nr > 0) switch (P.kmax) {
      case 1: klaunch(h, MVAMG_KC_PROLONG, pby, k_bprolong_rows<T, 1>, pg, kBlock, st, nr, P.nf, P.cinfo, tUrow<T>(P), xc, x); break;
      case 2: klaunch(h, MVAMG_KC_PROLONG, pby, k_bprolong_rows<T, 2>, pg, kBlock, st, nr, P.nf, P.cinfo, tUrow<T>(P), xc, x); break;
      case 3:
      case 4: klaunch(h, MVAMG_KC_PROLONG, pby, k_bprolong_rows<T, 4>, pg, kBlock, st, nr, P.nf, P.cinfo, tUrow<T>(P), xc, x); break;
      default: klaunch(h, MVAMG_KC_PROLONG, pby, k_bprolong_rows<T, 8>, pg, kBlock, st, nr, P.nf, P.cinfo, tUrow<T>(P), xc, x); break;
    }
  }
  LAUNCHCHECK("bprolong");
  if (smoother == MVAMG_SMOOTH_GS) {
    for (int c = L.ns - 1; c >= 0; --c) bgs_stage<T>(h, l, L, c, r, x, 1, st);
  } else {
    bresid<T, 0>(h, L, r, x, s, MM_STORE_R0, st);
    k_bl1_update<T><<<bgrid_elem(L.n), kBlock, 0, st>>>(L.n, ldl1<T>(L), s, x);
  }
  LAUNCHCHECK("bvcycle");
}

// Z = B R for level-0 binary64 block vectors in smoother order
void bapply_B(mvamg_hier* h, const double* r, double* z, int precision, int smoother, hipStream_t st,
              bool stage0_written = false) {
  if (precision == 64) {
    bvcycle<double>(h, 0, r, z, smoother, st, false, stage0_written);
  } else {
    DevLevel& L = h->lv[0];
    const int64_t m = (int64_t)L.n * kNB;
    k_cast<double, float><<<grid_elem(m), kBlock, 0, st>>>((int)m, r, L.br32);
    bvcycle<float>(h, 0, L.br32, L.bx32, smoother, st);
    k_cast<float, double><<<grid_elem(m), kBlock, 0, st>>>((int)m, L.bx32, z);
    LAUNCHCHECK("bapply_B32");
  }
}

// ---------------------------------------------------- multi-system CG

struct MultiOps {
  mvamg_hier* h = nullptr;
  int nsys = 0;   // systems carried on the device
  int nrep = 0;   // systems reported to the caller (the first nrep)
  int key = 0;    // graph cache key base
  const std::vector<char>* host_act = nullptr;  // host mirror of the systems' S_ACT flags
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  virtual ~MultiOps() {}
  virtual void load(const double* b, const double* x, hipStream_t st) = 0;  // caller layout -> internal
  virtual void store(double* x, hipStream_t st) = 0;
  virtual void resid(hipStream_t st) = 0;       // r = b - A x
  virtual void true_resid(hipStream_t st) = 0;  // q = b - A x, per-system q.q (MM_STORE_TRR)
  virtual void dot(const double* a, const double* b, const double* c, const double* d, int nv, int mode,
                   hipStream_t st) = 0;
  // the dot products inside an iteration (stopped systems may be skipped)
  virtual void dot_iter(const double* a, const double* b, const double* c, const double* d, int nv, int mode,
                        hipStream_t st) {
    dot(a, b, c, d, nv, mode, st);
  }
  // z = B r; after_update: r comes from this solve's last axpy2, which may
  // have written the first sweep stage of z already (see BlockOps)
  virtual void cycle(int precision, int smoother, hipStream_t st, bool after_update) = 0;
  int precision = 64, smoother = MVAMG_SMOOTH_GS;  // of the solve in progress
  virtual void copy_zp(hipStream_t st) = 0;
  virtual void spmv_pq(hipStream_t st) = 0;    // q = A p, per-system p.q (MM_PQ)
  virtual void axpy2(hipStream_t st) = 0;      // x += alpha p, r -= alpha q, per-system r.r (MM_STORE_RR)
  virtual void xpay(hipStream_t st) = 0;       // p = z + beta p
  // an x update that axpy2 defers to the next xpay, applied after the last step
  virtual void flush(hipStream_t) {}
};

void multi_step_a(MultiOps& O, hipStream_t st) {
  mvamg_hier* h = O.h;
  O.spmv_pq(st);
  O.axpy2(st);
  HIPCHECK(hipMemcpyAsync(h->mb.pinned, h->mb.scal, (size_t)O.nsys * S_NSCAL * sizeof(double),
                          hipMemcpyDeviceToHost, st));
}

void multi_step_b(MultiOps& O, int precision, int smoother, hipStream_t st) {
  O.cycle(precision, smoother, st, true);
  if (precision == 32)
    O.dot_iter(O.z, O.r, O.z, O.q, 2, MM_RZ_FLEX, st);
  else
    O.dot_iter(O.z, O.r, nullptr, nullptr, 1, MM_RZ, st);
  O.xpay(st);
}

hipGraphExec_t multi_graph(MultiOps& O, int precision, int smoother) {
  mvamg_hier* h = O.h;
  const int key = O.key + precision * 4 + smoother;
  auto it = h->graphs.find(key);
  if (it != h->graphs.end()) return it->second;
  if (!h->cap) HIPCHECK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  HIPCHECK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  try {
    multi_step_b(O, precision, smoother, h->cap);
    multi_step_a(O, h->cap);
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

void read_mscalars(mvamg_hier* h, int nsys, hipStream_t st) {
  HIPCHECK(hipMemcpyAsync(h->mb.pinned, h->mb.scal, (size_t)nsys * S_NSCAL * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
}

// S_ACT of every system from the host flags act (and S_FLAG cleared)
void upload_active(mvamg_hier* h, int nsys, const std::vector<char>& act, hipStream_t st) {
  MultiBufs& M = h->mb;
  HIPCHECK(hipStreamSynchronize(st));  // the pinned staging array may still be read by an earlier copy
  for (int s = 0; s < nsys; ++s) M.pact[s] = act[s] ? 1.0 : 0.0;
  HIPCHECK(hipMemcpyAsync(M.act, M.pact, (size_t)nsys * sizeof(double), hipMemcpyHostToDevice, st));
  k_mset_active<<<1, kBlock, 0, st>>>(nsys, M.act, M.scal);
  LAUNCHCHECK("mset_active");
}

// Preconditioned CG on every system at once.  Per system the sequence of
// operations is that of the single-system solve: the same stopping rule,
// iteration cap and (binary32 cycle) true-residual restarts; a system that
// stops keeps its iterate while the others go on.
mvamg_status multi_pcg(MultiOps& O, const double* b, double* x, const mvamg_solve_params* prm, mvamg_info* infos,
                       hipStream_t st) {
  mvamg_hier* h = O.h;
  if (!prm || !b || !x) throw Error(MVAMG_ERR_ARG, "null argument");
  if (prm->precision != 64 && prm->precision != 32) throw Error(MVAMG_ERR_ARG, "precision must be 64 or 32");
  if (prm->smoother != MVAMG_SMOOTH_GS && prm->smoother != MVAMG_SMOOTH_L1JACOBI)
    throw Error(MVAMG_ERR_ARG, "unknown smoother");
  if (prm->maxit < 0 || !(prm->rtol >= 0.0)) throw Error(MVAMG_ERR_ARG, "invalid maxit or rtol");
  const int ns = O.nsys;
  MultiBufs& M = h->mb;
  const double* pin = M.pinned;
  const bool flex = (prm->precision == 32);
  const int max_restarts = flex ? std::max(0, prm->max_restarts) : 0;
  const size_t hstride = (size_t)prm->maxit + 1;
  O.precision = prm->precision;
  O.smoother = prm->smoother;
  O.load(b, x, st);
  k_minit<<<1, kBlock, 0, st>>>(ns, M.scal, prm->rtol);
  LAUNCHCHECK("minit");
  O.resid(st);
  O.dot(O.r, O.r, nullptr, nullptr, 1, MM_STORE_R0, st);
  read_mscalars(h, ns, st);
  std::vector<double> r0(ns), hlast(ns, 1.0);
  std::vector<int> it(ns, 0), restarts(ns, 0);
  std::vector<char> run(ns, 0), met(ns, 0), conv(ns, 0), act(ns, 0);
  O.host_act = &act;
  for (int s = 0; s < ns; ++s) {
    r0[s] = std::sqrt(pin[s * S_NSCAL + S_R0]);
    if (!std::isfinite(r0[s]))
      throw Error(MVAMG_ERR_NONFINITE, "non-finite initial residual in system " + std::to_string(s));
    if (prm->history && s < O.nrep) prm->history[s * hstride] = 1.0;
    if (r0[s] == 0.0) {
      conv[s] = 1;
      hlast[s] = 0.0;
    } else {
      run[s] = prm->maxit > 0;
    }
  }
  bool first_round = true;
  auto any = [](const std::vector<char>& v) {
    for (char c : v)
      if (c) return true;
    return false;
  };
  while (any(run)) {
    if (!first_round) O.resid(st);
    act = run;
    for (int s = 0; s < ns; ++s)
      if (run[s]) met[s] = 0;
    upload_active(h, ns, act, st);
    O.cycle(prm->precision, prm->smoother, st, false);
    O.dot(O.r, O.z, nullptr, nullptr, 1, MM_RHO0, st);
    O.copy_zp(st);
    hipGraphExec_t ge = (h->use_graphs && !h->prof) ? multi_graph(O, prm->precision, prm->smoother) : nullptr;
    bool firstit = true;
    std::vector<char> was(ns);
    while (any(act)) {
      was = act;
      if (firstit) {
        multi_step_a(O, st);
        firstit = false;
      } else if (ge) {
        HIPCHECK(hipGraphLaunch(ge, st));
      } else {
        multi_step_b(O, prm->precision, prm->smoother, st);
        multi_step_a(O, st);
      }
      HIPCHECK(hipStreamSynchronize(st));
      bool changed = false;
      for (int s = 0; s < ns; ++s) {
        if (!was[s]) continue;
        const double* sc = pin + (size_t)s * S_NSCAL;
        it[s] += 1;
        if (sc[S_FLAG] != 0.0)
          throw Error(MVAMG_ERR_BREAKDOWN, "CG breakdown in system " + std::to_string(s) + ": p^T A p <= 0");
        const double hl = std::sqrt(sc[S_RR]) / r0[s];
        if (!std::isfinite(hl)) throw Error(MVAMG_ERR_NONFINITE, "non-finite residual in system " + std::to_string(s));
        hlast[s] = hl;
        if (prm->history && s < O.nrep) prm->history[s * hstride + it[s]] = hl;
        if (sc[S_ACT] == 0.0) {
          met[s] = 1;
          act[s] = 0;
        } else if (it[s] >= prm->maxit) {
          act[s] = 0;
          changed = true;
        }
      }
      if (changed && any(act)) upload_active(h, ns, act, st);
    }
    O.flush(st);
    if (!flex) {
      for (int s = 0; s < ns; ++s)
        if (run[s]) {
          conv[s] = met[s];
          run[s] = 0;
        }
    } else {
      O.true_resid(st);
      read_mscalars(h, ns, st);
      for (int s = 0; s < ns; ++s) {
        if (!run[s]) continue;
        const double tr = std::sqrt(pin[s * S_NSCAL + S_TRR]) / r0[s];
        if (met[s] && tr <= prm->rtol) {
          conv[s] = 1;
          run[s] = 0;
        } else if (restarts[s] < max_restarts && it[s] < prm->maxit) {
          restarts[s] += 1;
        } else {
          run[s] = 0;
        }
      }
    }
    first_round = false;
  }
  // true residuals and the iterates in the caller's layout
  O.true_resid(st);
  O.store(x, st);
  read_mscalars(h, ns, st);
  bool all = true;
  for (int s = 0; s < O.nrep; ++s) {
    all = all && conv[s];
    if (infos) {
      mvamg_info& inf = infos[s];
      inf.iterations = it[s];
      inf.converged = conv[s];
      inf.restarts = restarts[s];
      inf.rel_res = hlast[s];
      inf.rel_res_true = (r0[s] > 0.0) ? std::sqrt(pin[s * S_NSCAL + S_TRR]) / r0[s] : 0.0;
    }
  }
  if (h->prof) harvest(h);
  return all ? MVAMG_OK : MVAMG_NOT_CONVERGED;
}

// ------------------------------------------------------- block columns

struct BlockOps : MultiOps {
  int m = 0;  // caller's columns (<= 32); columns m..31 are zero and stopped
  BlockOps(mvamg_hier* hh, int mm) {
    h = hh;
    m = mm;
    nsys = kNB;
    nrep = mm;
    key = 1000;
    r = h->lv[0].br;
    z = h->lv[0].bx;
    p = h->bp;
    q = h->bq;
  }
  int n() const { return h->n; }
  void load(const double* b, const double* x, hipStream_t st) override {
    k_bgather<<<bgrid_elem(n()), kBlock, 0, st>>>(n(), h->perm0, m, b, h->bb);
    k_bgather<<<bgrid_elem(n()), kBlock, 0, st>>>(n(), h->perm0, m, x, h->bxv);
    LAUNCHCHECK("bgather");
  }
  void store(double* x, hipStream_t st) override {
    k_bscatter<<<bgrid_elem(n()), kBlock, 0, st>>>(n(), h->perm0, m, h->bxv, x);
    LAUNCHCHECK("bscatter");
  }
  void resid(hipStream_t st) override { bresid<double, 0>(h, h->lv[0], h->bb, h->bxv, r, MM_STORE_R0, st); }
  void true_resid(hipStream_t st) override {
    bresid<double, 0>(h, h->lv[0], h->bb, h->bxv, q, MM_STORE_R0, st);
    dot(q, q, nullptr, nullptr, 1, MM_STORE_TRR, st);
  }
  void dot(const double* a, const double* b, const double* c, const double* d, int nv, int mode,
           hipStream_t st) override {
    const int grid = bgrid_for(n());
    if (nv == 1) {
      k_bdot<1><<<grid, kBlock, 0, st>>>(n(), a, b, nullptr, nullptr, h->mb.part);
      k_mfinish<1><<<kNB, kBlock, 0, st>>>(kNB, grid, h->mb.part, h->mb.scal, mode);
    } else {
      k_bdot<2><<<grid, kBlock, 0, st>>>(n(), a, b, c, d, h->mb.part);
      k_mfinish<2><<<kNB, kBlock, 0, st>>>(kNB, grid, h->mb.part, h->mb.scal, mode);
    }
    LAUNCHCHECK("bdot");
  }
  // The binary64 Gauss-Seidel cycle on a point fine level starts with z = r / d
  // on stage 0; the residual update writes those rows with the new r.
  bool fuse_stage0() const {
    return precision == 64 && smoother == MVAMG_SMOOTH_GS && h->lv[0].sell && h->nl > 1;
  }
  void cycle(int prec, int sm, hipStream_t st, bool after_update) override {
    bapply_B(h, r, z, prec, sm, st, after_update && fuse_stage0());
  }
  void copy_zp(hipStream_t st) override {
    const int64_t e = (int64_t)n() * kNB;
    k_copy<double><<<grid_elem(e), kBlock, 0, st>>>((int)e, z, p);
    LAUNCHCHECK("bcopy");
  }
  void spmv_pq(hipStream_t st) override { bresid<double, 1>(h, h->lv[0], nullptr, p, q, MM_PQ, st); }
  // r -= alpha q now; x += alpha p with the next p update (or flush)
  void axpy2(hipStream_t st) override {
    const int grid = bgrid_for(n());
    const DevLevel& L = h->lv[0];
    k_br_update_dot<<<grid, kBlock, 0, st>>>(n(), h->mb.scal, q, r, h->mb.part, fuse_stage0() ? L.rows0 : 0,
                                             ldblk<double>(L), z);
    k_mfinish<1><<<kNB, kBlock, 0, st>>>(kNB, grid, h->mb.part, h->mb.scal, MM_STORE_RR);
    LAUNCHCHECK("br_update");
  }
  void xpay(hipStream_t st) override {
    k_bxpay<<<bgrid_elem(n()), kBlock, 0, st>>>(n(), h->mb.scal, z, p, h->bxv);
    LAUNCHCHECK("bxpay");
  }
  void flush(hipStream_t st) override {
    k_bx_update<<<bgrid_elem(n()), kBlock, 0, st>>>(n(), h->mb.scal, p, h->bxv);
    LAUNCHCHECK("bx_update");
  }
};

// ------------------------------------------------- batch of problems

// Inside the CG iterations the work of problems that have stopped is skipped
// (level-0 kernels and the per-problem vector kernels); their iterates and
// residuals stay as they were, exactly as for a problem solved on its own.
struct BatchOps : MultiOps {
  explicit BatchOps(mvamg_hier* hh) {
    h = hh;
    nsys = hh->nprob;
    nrep = hh->nprob;
    key = 2000;
    r = h->r;
    z = h->z;
    p = h->p;
    q = h->q;
  }
  struct SkipScope {  // level-0 kernels skip stopped problems while alive
    mvamg_hier* h;
    SkipScope(mvamg_hier* hh, const std::vector<char>* act) : h(hh) {
      h->skip_act = h->mb.scal + S_ACT;
      double rows = 0.0;
      for (int p = 0; p < h->nprob; ++p)
        if (!act || (*act)[p]) rows += h->h_poff[p + 1] - h->h_poff[p];
      h->skip_frac = rows / std::max(1, h->n);
    }
    ~SkipScope() {
      h->skip_act = nullptr;
      h->skip_frac = 1.0;
    }
  };
  const double* act() const { return h->mb.scal + S_ACT; }
  dim3 pgrid() const { return dim3(h->pchunks, h->nprob); }
  // with problems on the small-problem path, the caller's vectors hold every
  // problem: umap takes a row of this part to the caller's row
  void load(const double* b, const double* x, hipStream_t st) override {
    if (h->umap) {
      k_gather2<<<grid_for(h->n), kBlock, 0, st>>>(h->n, h->perm0, h->umap, b, h->b);
      k_gather2<<<grid_for(h->n), kBlock, 0, st>>>(h->n, h->perm0, h->umap, x, h->x);
    } else {
      k_gather<<<grid_for(h->n), kBlock, 0, st>>>(h->n, h->perm0, b, h->b);
      k_gather<<<grid_for(h->n), kBlock, 0, st>>>(h->n, h->perm0, x, h->x);
    }
    LAUNCHCHECK("gather");
  }
  void store(double* x, hipStream_t st) override {
    if (h->umap)
      k_scatter2<<<grid_for(h->n), kBlock, 0, st>>>(h->n, h->perm0, h->umap, h->x, x);
    else
      k_scatter<<<grid_for(h->n), kBlock, 0, st>>>(h->n, h->perm0, h->x, x);
    LAUNCHCHECK("scatter");
  }
  void resid(hipStream_t st) override { ::resid<double, 0>(h, 0, h->lv[0], h->b, h->x, r, M_NONE, st); }
  void true_resid(hipStream_t st) override {
    ::resid<double, 0>(h, 0, h->lv[0], h->b, h->x, q, M_NONE, st);
    dot(q, q, nullptr, nullptr, 1, MM_STORE_TRR, st);
  }
  void pdot(const double* a, const double* b, const double* c, const double* d, int nv, int mode,
            const double* skip, hipStream_t st) {
    if (nv == 1) {
      k_pdot<1><<<pgrid(), kBlock, 0, st>>>(h->poff, h->iperm0, a, b, nullptr, nullptr, h->mb.part, skip);
      k_mfinish<1><<<h->nprob, kBlock, 0, st>>>(h->nprob, h->pchunks, h->mb.part, h->mb.scal, mode);
    } else {
      k_pdot<2><<<pgrid(), kBlock, 0, st>>>(h->poff, h->iperm0, a, b, c, d, h->mb.part, skip);
      k_mfinish<2><<<h->nprob, kBlock, 0, st>>>(h->nprob, h->pchunks, h->mb.part, h->mb.scal, mode);
    }
    LAUNCHCHECK("pdot");
  }
  void dot(const double* a, const double* b, const double* c, const double* d, int nv, int mode,
           hipStream_t st) override {
    pdot(a, b, c, d, nv, mode, nullptr, st);
  }
  void dot_iter(const double* a, const double* b, const double* c, const double* d, int nv, int mode,
                hipStream_t st) override {
    pdot(a, b, c, d, nv, mode, act(), st);
  }
  void cycle(int prec, int sm, hipStream_t st, bool) override {
    SkipScope sk(h, host_act);
    apply_B(h, r, z, prec, sm, st);
  }
  void copy_zp(hipStream_t st) override {
    k_copy<double><<<grid_elem(h->n), kBlock, 0, st>>>(h->n, z, p);
    LAUNCHCHECK("copy");
  }
  void spmv_pq(hipStream_t st) override {
    {
      SkipScope sk(h, host_act);
      ::resid<double, 2>(h, 0, h->lv[0], nullptr, p, q, M_NONE, st);
    }
    dot_iter(p, q, nullptr, nullptr, 1, MM_PQ, st);
  }
  void axpy2(hipStream_t st) override {
    k_paxpy2_dot<<<pgrid(), kBlock, 0, st>>>(h->poff, h->iperm0, h->mb.scal, p, q, h->x, r, h->mb.part, 1);
    k_mfinish<1><<<h->nprob, kBlock, 0, st>>>(h->nprob, h->pchunks, h->mb.part, h->mb.scal, MM_STORE_RR);
    LAUNCHCHECK("paxpy2");
  }
  void xpay(hipStream_t st) override {
    k_pxpay<<<pgrid(), kBlock, 0, st>>>(h->poff, h->iperm0, h->mb.scal, z, p, 1);
    LAUNCHCHECK("pxpay");
  }
};
