// Small problems of a batch in one persistent launch: one workgroup solves a
// whole problem -- preconditioned CG (Section 5) with its own V-cycle over its
// own hierarchy, any number of levels -- using only workgroup barriers.  The
// workgroups stride over the problems.  Layout per level (the problem's
// smoother order): CSR with the diagonal kept separately, smoother stages as
// runs of groups, groups as runs of rows; transfers per aggregate (members,
// coarse dofs, U_a row-major n_a x k_a); the coarsest inverse dense.
#pragma once

#include "kernels.hpp"
#include "mvamg.h"

namespace mvamg {

constexpr int kMiniBlock = 1024;
constexpr int kMiniMaxLevels = 16;
constexpr int kMiniMaxIt = 1000;  // history slots per problem

struct MiniLevel {
  int n, ns;          // rows; smoother stages (0 on the coarsest)
  int64_t rp, ci;     // ints: row pointers (n + 1, relative to ci), column indices
  int64_t va, dg;     // reals: values (CSR order), diagonal (n)
  int64_t dl;         // reals: l1 row norms (n)
  int64_t sgrp, gptr; // ints: stage -> first group (ns + 1), group -> first row
  int nagg;           // aggregates of the transfer to the next level (0 on the coarsest)
  int64_t aptr, arows, cptr, cdof, uoff;  // ints: members, coarse dofs (next level's numbering), U offsets
  int64_t U;          // reals: U_a blocks, row-major n_a x k_a
  int64_t r, x, s;    // work: the level's right-hand side, iterate, residual
};

struct MiniProb {
  int nl, lev0, n;    // levels, first MiniLevel, fine rows
  int64_t perm0;      // ints: smoother order -> the problem's rows
  int64_t ainv;       // reals: coarsest inverse (n_L x n_L, entry (i, j) at j n_L + i)
  int64_t row0;       // first row of the problem in the batch vectors
  int64_t cr, cz, cp, cq, cx;  // work: the CG vectors (n)
};

struct MiniInfo {
  int iterations, converged, status;  // status: 0 ok, 1 not converged, -5 breakdown, -4 non-finite
  double rel_res, rel_res_true;
};

// Sum over the workgroup in a fixed order; every thread gets the result.
__device__ __forceinline__ double mini_sum(double v, double* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < kMiniBlock / 64; ++q) t += lds[q];
  return t;
}

// y = A x (level L) or, with r, y = r - A x
__device__ __forceinline__ void mini_apply(const MiniLevel& L, const int* I, const double* D, const double* r,
                                           const double* x, double* y) {
  const int* rp = I + L.rp;
  const int* ci = I + L.ci;
  const double* va = D + L.va;
  for (int i = threadIdx.x; i < L.n; i += kMiniBlock) {
    double s = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) s += va[e] * x[ci[e]];
    y[i] = r ? r[i] - s : s;
  }
}

// One Gauss-Seidel relaxation of row i: x_i <- (r_i - sum_{j != i} a_ij x_j) / a_ii
__device__ __forceinline__ void mini_gs_row(const int* rp, const int* ci, const double* va, const double* dg,
                                            const double* r, double* x, int i) {
  double s = r[i];
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const int j = ci[e];
    if (j != i) s -= va[e] * x[j];
  }
  x[i] = s / dg[i];
}

// One sweep in the level's order (forward) or the reverse order (backward);
// the groups of a stage are independent, a group's rows go one after another.
__device__ void mini_gs(const MiniLevel& L, const int* I, const double* D, const double* r, double* x,
                        bool forward) {
  const int* rp = I + L.rp;
  const int* ci = I + L.ci;
  const double* va = D + L.va;
  const double* dg = D + L.dg;
  const int* sgrp = I + L.sgrp;
  const int* gptr = I + L.gptr;
  for (int cc = 0; cc < L.ns; ++cc) {
    const int c = forward ? cc : L.ns - 1 - cc;
    for (int g = sgrp[c] + threadIdx.x; g < sgrp[c + 1]; g += kMiniBlock) {
      if (forward)
        for (int i = gptr[g]; i < gptr[g + 1]; ++i) mini_gs_row(rp, ci, va, dg, r, x, i);
      else
        for (int i = gptr[g + 1] - 1; i >= gptr[g]; --i) mini_gs_row(rp, ci, va, dg, r, x, i);
    }
    __syncthreads();
  }
}

// x <- x + D_l1^{-1} (r - A x) (Baker, Falgout, Kolev, Yang 2011), s scratch
__device__ void mini_l1(const MiniLevel& L, const int* I, const double* D, const double* r, double* x, double* s) {
  mini_apply(L, I, D, r, x, s);
  __syncthreads();
  const double* dl = D + L.dl;
  for (int i = threadIdx.x; i < L.n; i += kMiniBlock) x[i] = x[i] + s[i] / dl[i];
  __syncthreads();
}

// z = B r: one V-cycle over the problem's levels (r, z: level 0 vectors)
__device__ void mini_vcycle(const MiniProb& P, const MiniLevel* lev, const int* I, const double* D, double* W,
                            const double* r0, double* z0, int smoother) {
  const int nl = P.nl;
  for (int l = 0; l < nl - 1; ++l) {
    const MiniLevel& L = lev[l];
    const double* r = l == 0 ? r0 : W + L.r;
    double* x = l == 0 ? z0 : W + L.x;
    double* s = W + L.s;
    for (int i = threadIdx.x; i < L.n; i += kMiniBlock) x[i] = 0.0;
    __syncthreads();
    if (smoother == MVAMG_SMOOTH_GS)
      mini_gs(L, I, D, r, x, true);
    else
      mini_l1(L, I, D, r, x, s);
    mini_apply(L, I, D, r, x, s);
    __syncthreads();
    // r_{l+1}[coarse dof m of a] = sum over members q of U_a[q][m] s[member q]
    const MiniLevel& C = lev[l + 1];
    double* rc = W + C.r;
    const int* aptr = I + L.aptr;
    const int* arows = I + L.arows;
    const int* cptr = I + L.cptr;
    const int* cdof = I + L.cdof;
    const int* uoff = I + L.uoff;
    const double* U = D + L.U;
    for (int a = threadIdx.x; a < L.nagg; a += kMiniBlock) {
      const int k = cptr[a + 1] - cptr[a];
      for (int m = 0; m < k; ++m) {
        double acc = 0.0;
        for (int q = aptr[a]; q < aptr[a + 1]; ++q) acc += U[uoff[a] + (q - aptr[a]) * k + m] * s[arows[q]];
        rc[cdof[cptr[a] + m]] = acc;
      }
    }
    __syncthreads();
  }
  {
    // coarsest: x = A_L^{-1} r
    const MiniLevel& C = lev[nl - 1];
    const double* rc = W + C.r;
    double* xc = W + C.x;
    const double* Ai = D + P.ainv;
    // the inverse is stored column by column (entry (i, j) at j n + i), so
    // the threads' reads of one j are adjacent
    for (int i = threadIdx.x; i < C.n; i += kMiniBlock) {
      double acc = 0.0;
      for (int j = 0; j < C.n; ++j) acc += Ai[(int64_t)j * C.n + i] * rc[j];
      xc[i] = acc;
    }
    __syncthreads();
  }
  for (int l = nl - 2; l >= 0; --l) {
    const MiniLevel& L = lev[l];
    const MiniLevel& C = lev[l + 1];
    const double* r = l == 0 ? r0 : W + L.r;
    double* x = l == 0 ? z0 : W + L.x;
    const double* xc = W + C.x;
    const int* aptr = I + L.aptr;
    const int* arows = I + L.arows;
    const int* cptr = I + L.cptr;
    const int* cdof = I + L.cdof;
    const int* uoff = I + L.uoff;
    const double* U = D + L.U;
    // x += P x_c: every row belongs to one aggregate
    for (int a = threadIdx.x; a < L.nagg; a += kMiniBlock) {
      const int k = cptr[a + 1] - cptr[a];
      for (int q = aptr[a]; q < aptr[a + 1]; ++q) {
        double acc = 0.0;
        for (int m = 0; m < k; ++m) acc += U[uoff[a] + (q - aptr[a]) * k + m] * xc[cdof[cptr[a] + m]];
        x[arows[q]] += acc;
      }
    }
    __syncthreads();
    if (smoother == MVAMG_SMOOTH_GS)
      mini_gs(L, I, D, r, x, false);
    else
      mini_l1(L, I, D, r, x, W + L.s);
  }
}

// Preconditioned CG on every problem (x: initial guesses in, solutions out;
// both in the batch's row order); per problem its own stopping test.
__global__ __launch_bounds__(kMiniBlock) void k_mini_pcg(int nprob, const MiniProb* __restrict__ probs,
                                                         const MiniLevel* __restrict__ levs, const int* I,
                                                         const double* D, double* W, const double* b, double* xio,
                                                         double rtol, int maxit, int smoother, double* hist,
                                                         MiniInfo* info) {
  __shared__ double lds[kMiniBlock / 64];
  for (int pi = blockIdx.x; pi < nprob; pi += gridDim.x) {
    const MiniProb P = probs[pi];
    const MiniLevel* lev = levs + P.lev0;
    const MiniLevel& L0 = lev[0];
    const int n = P.n;
    const int* perm = I + P.perm0;
    double *r = W + P.cr, *z = W + P.cz, *p = W + P.cp, *q = W + P.cq, *x = W + P.cx;
    double* h = hist ? hist + (int64_t)pi * (kMiniMaxIt + 1) : nullptr;  // maxit <= kMiniMaxIt
    for (int i = threadIdx.x; i < n; i += kMiniBlock) {
      x[i] = xio[P.row0 + perm[i]];
      z[i] = b[P.row0 + perm[i]];
    }
    __syncthreads();
    mini_apply(L0, I, D, z, x, r);  // r = b - A x
    __syncthreads();
    double rr = 0.0;
    for (int i = threadIdx.x; i < n; i += kMiniBlock) rr += r[i] * r[i];
    const double r0 = sqrt(mini_sum(rr, lds));
    MiniInfo inf{0, 0, 1, 1.0, 0.0};
    if (h && threadIdx.x == 0) h[0] = 1.0;
    if (!isfinite(r0)) {
      inf.status = -4;
    } else if (r0 == 0.0) {
      inf.status = 0;
      inf.converged = 1;
      inf.rel_res = 0.0;
    } else {
      mini_vcycle(P, lev, I, D, W, r, z, smoother);
      double rz = 0.0;
      for (int i = threadIdx.x; i < n; i += kMiniBlock) {
        p[i] = z[i];
        rz += r[i] * z[i];
      }
      double rho = mini_sum(rz, lds);
      for (int it = 0; it < maxit; ++it) {
        mini_apply(L0, I, D, nullptr, p, q);
        __syncthreads();
        double pq = 0.0;
        for (int i = threadIdx.x; i < n; i += kMiniBlock) pq += p[i] * q[i];
        pq = mini_sum(pq, lds);
        if (!(pq > 0.0)) {
          inf.status = -5;
          break;
        }
        const double alpha = rho / pq;
        double rr2 = 0.0;
        for (int i = threadIdx.x; i < n; i += kMiniBlock) {
          x[i] += alpha * p[i];
          r[i] -= alpha * q[i];
          rr2 += r[i] * r[i];
        }
        const double hk = sqrt(mini_sum(rr2, lds)) / r0;
        inf.iterations = it + 1;
        inf.rel_res = hk;
        if (h && threadIdx.x == 0) h[it + 1] = hk;
        if (!isfinite(hk)) {
          inf.status = -4;
          break;
        }
        if (hk <= rtol) {
          inf.status = 0;
          inf.converged = 1;
          break;
        }
        mini_vcycle(P, lev, I, D, W, r, z, smoother);
        double rz2 = 0.0;
        for (int i = threadIdx.x; i < n; i += kMiniBlock) rz2 += r[i] * z[i];
        const double rho2 = mini_sum(rz2, lds);
        const double beta = rho2 / rho;
        rho = rho2;
        for (int i = threadIdx.x; i < n; i += kMiniBlock) p[i] = z[i] + beta * p[i];
        __syncthreads();
      }
    }
    // true residual and the solution back in the batch's row order
    for (int i = threadIdx.x; i < n; i += kMiniBlock) z[i] = b[P.row0 + perm[i]];
    __syncthreads();
    mini_apply(L0, I, D, z, x, q);
    __syncthreads();
    double tr = 0.0;
    for (int i = threadIdx.x; i < n; i += kMiniBlock) {
      tr += q[i] * q[i];
      xio[P.row0 + perm[i]] = x[i];
    }
    tr = mini_sum(tr, lds);
    inf.rel_res_true = r0 > 0.0 ? sqrt(tr) / r0 : 0.0;
    if (threadIdx.x == 0) info[pi] = inf;
    __syncthreads();
  }
}

}  // namespace mvamg
