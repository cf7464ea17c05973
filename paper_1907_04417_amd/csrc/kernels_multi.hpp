// Device kernels for many systems at once: several right-hand sides through
// one hierarchy, and several independent problems solved together.
//
// Block vectors (several right-hand sides): n x 32 row-major, row i holding
// the 32 values x[i * 32 + c], so one matrix entry, loaded once, multiplies a
// contiguous 256-byte row (binary64) of the block.  A half wavefront (32
// lanes) owns one matrix row, lane c its column c.
//
// Every system s (a column, or a problem) runs its own conjugate-gradient
// recurrence: its scalars sit at scal[s * S_NSCAL + k] and a per-system flag
// S_ACT stops its updates once its residual met the tolerance.
#pragma once

#include <type_traits>

#include "kernels.hpp"

namespace mvamg {

constexpr int kNB = 32;  // columns of a block vector

// per-system scalars beyond those of a single system
enum MScalar { S_ACT = 8, S_RTOL = 9, S_R0N = 10, S_TRR = 11 };

enum MMode {
  MM_STORE_R0 = 0,  // ||r_0||^2 and its root
  MM_STORE_RR = 1,  // r.r after an update; clears S_ACT once ||r|| / ||r_0|| <= rtol
  MM_STORE_TRR = 2, // ||b - A x||^2 recomputed
  MM_PQ = 3,        // p.A p and alpha (zero for stopped systems)
  MM_RHO0 = 4,      // r.z at a (re)start
  MM_RZ = 5,        // r.z and beta (zero for stopped systems)
  MM_RZ_FLEX = 6    // r.z, z.q and the flexible beta
};

__device__ __forceinline__ void mepilogue(int mode, double v0, double v1, double* sc) {
  const bool act = sc[S_ACT] != 0.0;
  switch (mode) {
    case MM_STORE_R0:
      sc[S_R0] = v0;
      sc[S_R0N] = sqrt(v0);
      break;
    case MM_STORE_RR:
      sc[S_RR] = v0;
      if (act && sqrt(v0) / sc[S_R0N] <= sc[S_RTOL]) sc[S_ACT] = 0.0;
      break;
    case MM_STORE_TRR: sc[S_TRR] = v0; break;
    case MM_PQ:
      if (act) {
        sc[S_PQ] = v0;
        if (!(v0 > 0.0)) sc[S_FLAG] = 1.0;
        sc[S_ALPHA] = sc[S_RHO] / v0;
      } else {
        sc[S_ALPHA] = 0.0;
      }
      break;
    case MM_RHO0: sc[S_RHO] = v0; break;
    case MM_RZ:
      sc[S_BETA] = act ? v0 / sc[S_RHO] : 0.0;
      sc[S_RHO] = v0;
      break;
    case MM_RZ_FLEX:
      if (act) {
        sc[S_ZQ] = v1;
        sc[S_BETA] = -sc[S_ALPHA] * v1 / sc[S_RHO];
      } else {
        sc[S_BETA] = 0.0;
      }
      sc[S_RHO] = v0;
      break;
  }
}

// all scalars zero, S_RTOL = rtol
__global__ __launch_bounds__(kBlock) void k_minit(int nsys, double* scal, double rtol) {
  for (int i = threadIdx.x; i < nsys * S_NSCAL; i += kBlock) scal[i] = ((i % S_NSCAL) == S_RTOL) ? rtol : 0.0;
}

// S_ACT of every system from act[s] (0 or 1); S_FLAG cleared
__global__ __launch_bounds__(kBlock) void k_mset_active(int nsys, const double* __restrict__ act, double* scal) {
  for (int s = threadIdx.x; s < nsys; s += kBlock) {
    scal[s * S_NSCAL + S_ACT] = act[s];
    scal[s * S_NSCAL + S_FLAG] = 0.0;
  }
}

// Block s adds the partials part[(v * nsys + s) * nparts + b] in order b =
// 0, 1, ... and applies the epilogue of system s.
template <int NV>
__global__ __launch_bounds__(kBlock) void k_mfinish(int nsys, int nparts, const double* __restrict__ part,
                                                    double* scal, int mode) {
  __shared__ double lds[4];
  const int s = blockIdx.x;
  const double* p0 = part + (size_t)s * nparts;
  const double* p1 = part + (size_t)(nsys + s) * nparts;
  double s0 = 0.0, s1 = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) {
    s0 += p0[i];
    if (NV > 1) s1 += p1[i];
  }
  s0 = block_sum(s0, lds);
  if (NV > 1) s1 = block_sum(s1, lds);
  if (threadIdx.x == 0) mepilogue(mode, s0, s1, scal + (size_t)s * S_NSCAL);
}

// ------------------------------------------------- block-vector kernels

// Per-column sums over a 256-thread block whose lane c (threadIdx & 31) holds
// column c: part[(v * 32 + c) * gridDim.x + blockIdx.x].  Every thread of the
// block must call it.
__device__ __forceinline__ void bcol_partials(double a, int v, double* part) {
  __shared__ double lds[4][kNB];
  a += __shfl_xor(a, 32, 64);
  const int w = threadIdx.x >> 6, c = threadIdx.x & 31;
  if ((threadIdx.x & 63) < 32) lds[w][c] = a;
  __syncthreads();
  if (threadIdx.x < 32)
    part[(size_t)(v * kNB + c) * gridDim.x + blockIdx.x] = ((lds[0][c] + lds[1][c]) + lds[2][c]) + lds[3][c];
  __syncthreads();
}

// rows handled per 256-thread block and step of a row-per-half-wave loop
constexpr int kRowsPerBlock = kBlock / kNB;

// out[p][c] = in[perm[p]][c] for c < m (in: n x m row-major), 0 for c >= m
__global__ __launch_bounds__(kBlock) void k_bgather(int n, const int* __restrict__ perm, int m,
                                                    const double* __restrict__ in, double* __restrict__ out) {
  const int c = threadIdx.x & 31;
  for (int p = (blockIdx.x * kBlock + threadIdx.x) >> 5; p < n; p += gridDim.x * kRowsPerBlock)
    out[(size_t)p * kNB + c] = (c < m) ? in[(size_t)perm[p] * m + c] : 0.0;
}

// out[perm[p]][c] = in[p][c] for c < m
__global__ __launch_bounds__(kBlock) void k_bscatter(int n, const int* __restrict__ perm, int m,
                                                     const double* __restrict__ in, double* __restrict__ out) {
  const int c = threadIdx.x & 31;
  for (int p = (blockIdx.x * kBlock + threadIdx.x) >> 5; p < n; p += gridDim.x * kRowsPerBlock)
    if (c < m) out[(size_t)perm[p] * m + c] = in[(size_t)p * kNB + c];
}

// per-column a.b (and c.d)
template <int NV>
__global__ __launch_bounds__(kBlock) void k_bdot(int n, const double* __restrict__ a, const double* __restrict__ b,
                                                 const double* __restrict__ c2, const double* __restrict__ d,
                                                 double* __restrict__ part) {
  const int c = threadIdx.x & 31;
  double s0 = 0.0, s1 = 0.0;
  for (int p = (blockIdx.x * kBlock + threadIdx.x) >> 5; p < n; p += gridDim.x * kRowsPerBlock) {
    const size_t i = (size_t)p * kNB + c;
    s0 += a[i] * b[i];
    if (NV > 1) s1 += c2[i] * d[i];
  }
  bcol_partials(s0, 0, part);
  if (NV > 1) bcol_partials(s1, 1, part);
}

// columns still running: r -= alpha_c q; per-column r.r.  The matching
// x += alpha_c p is deferred to the next p update (k_bxpay), which reads p
// anyway, or to k_bx_update after the last step: alpha stays in the column's
// scalars until the next p.A p replaces it (with zero once the column has
// stopped), so no update is lost or applied twice.
// rows0 > 0: also the first stage of the next cycle's forward sweep from
// zero on a point fine level, z = r / d on the rows below rows0 (as
// k_bstage0_point, from the new r).
__global__ __launch_bounds__(kBlock) void k_br_update_dot(int n, const double* __restrict__ scal,
                                                          const double* __restrict__ q, double* __restrict__ r,
                                                          double* __restrict__ part, int rows0,
                                                          const double* __restrict__ diag, double* __restrict__ z) {
  const int c = threadIdx.x & 31;
  const double alpha = scal[c * S_NSCAL + S_ALPHA];
  const bool act = scal[c * S_NSCAL + S_ACT] != 0.0;
  double s = 0.0;
  for (int row = (blockIdx.x * kBlock + threadIdx.x) >> 5; row < n; row += gridDim.x * kRowsPerBlock) {
    const size_t i = (size_t)row * kNB + c;
    double ri = r[i];
    if (act) {
      ri -= alpha * q[i];
      r[i] = ri;
    }
    s += ri * ri;
    if (row < rows0) z[i] = ri / diag[row];
  }
  bcol_partials(s, 0, part);
}

// x += alpha_c p (the previous step's, deferred), then p = z + beta_c p
__global__ __launch_bounds__(kBlock) void k_bxpay(int n, const double* __restrict__ scal,
                                                  const double* __restrict__ z, double* __restrict__ p,
                                                  double* __restrict__ x) {
  const int c = threadIdx.x & 31;
  const double beta = scal[c * S_NSCAL + S_BETA], alpha = scal[c * S_NSCAL + S_ALPHA];
  for (int row = (blockIdx.x * kBlock + threadIdx.x) >> 5; row < n; row += gridDim.x * kRowsPerBlock) {
    const size_t i = (size_t)row * kNB + c;
    const double pi = p[i];
    x[i] += alpha * pi;
    p[i] = z[i] + beta * pi;
  }
}

// x += alpha_c p: the deferred update of the last step
__global__ __launch_bounds__(kBlock) void k_bx_update(int n, const double* __restrict__ scal,
                                                      const double* __restrict__ p, double* __restrict__ x) {
  const int c = threadIdx.x & 31;
  const double alpha = scal[c * S_NSCAL + S_ALPHA];
  for (int row = (blockIdx.x * kBlock + threadIdx.x) >> 5; row < n; row += gridDim.x * kRowsPerBlock) {
    const size_t i = (size_t)row * kNB + c;
    x[i] += alpha * p[i];
  }
}

// Lane J of each 32-lane half wave, broadcast to the half wave (ds_swizzle
// in bit mode: and-mask 0, or-mask J).
template <int J>
__device__ __forceinline__ int half_bcast(int v) {
  return __builtin_amdgcn_ds_swizzle(v, J << 5);
}
template <int J>
__device__ __forceinline__ double half_bcast(double v) {
  return __hiloint2double(half_bcast<J>(__double2hiint(v)), half_bcast<J>(__double2loint(v)));
}
template <int J>
__device__ __forceinline__ float half_bcast(float v) {
  return __int_as_float(half_bcast<J>(__float_as_int(v)));
}

// Entries J0 .. J0 + 7 of a half wave's row, whose lane c holds entry c of
// the current 32-entry chunk (mc, mv), broadcast to every lane.
template <int J0, typename T>
__device__ __forceinline__ void half_entries8(int mc, T mv, int (&cc)[8], T (&vv)[8]) {
  cc[0] = half_bcast<J0 + 0>(mc); vv[0] = half_bcast<J0 + 0>(mv);
  cc[1] = half_bcast<J0 + 1>(mc); vv[1] = half_bcast<J0 + 1>(mv);
  cc[2] = half_bcast<J0 + 2>(mc); vv[2] = half_bcast<J0 + 2>(mv);
  cc[3] = half_bcast<J0 + 3>(mc); vv[3] = half_bcast<J0 + 3>(mv);
  cc[4] = half_bcast<J0 + 4>(mc); vv[4] = half_bcast<J0 + 4>(mv);
  cc[5] = half_bcast<J0 + 5>(mc); vv[5] = half_bcast<J0 + 5>(mv);
  cc[6] = half_bcast<J0 + 6>(mc); vv[6] = half_bcast<J0 + 6>(mv);
  cc[7] = half_bcast<J0 + 7>(mc); vv[7] = half_bcast<J0 + 7>(mv);
}

// acc + SGN * (sum over the row's entries (col, val at cp[64 j], vp[64 j],
// j < width) of val * x[col * kNB + c]), the terms added one after the other;
// entries with col >= lim are skipped (forward sweep from zero).  Lane c loads
// entry j0 + c of each 32-entry chunk once; the entries reach the other lanes
// by swizzle.  The eight neighbour rows of a step are requested together with
// in-range indices, and a skipped term is a zero weight (a select, not a
// branch), so no wait sits between the requests.
template <typename T, int SGN>
__device__ __forceinline__ T half_row_sum(T acc, const int* __restrict__ cp, const T* __restrict__ vp, int width,
                                          int c, const T* x, int lim) {
  for (int j0 = 0; j0 < width; j0 += 32) {
    const int jc = min(j0 + c, width - 1);
    const int mc = cp[64 * jc];
    const T mv = vp[64 * jc];
    auto step = [&](auto J0c) {
      constexpr int J0 = decltype(J0c)::value;
      if (j0 + J0 < width) {
        int cc[8];
        T vv[8], xx[8];
        half_entries8<J0>(mc, mv, cc, vv);
#pragma unroll
        for (int u = 0; u < 8; ++u) xx[u] = x[(size_t)min(cc[u], lim - 1) * kNB + c];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          // a skipped term adds a zero product (xx is a finite value of a
          // row that is set: the index was clamped into range)
          const T w = ((j0 + J0 + u < width) & (cc[u] < lim)) ? vv[u] : T(0);
          if (SGN > 0)
            acc += w * xx[u];
          else
            acc -= w * xx[u];
        }
      }
    };
    step(std::integral_constant<int, 0>{});
    step(std::integral_constant<int, 8>{});
    step(std::integral_constant<int, 16>{});
    step(std::integral_constant<int, 24>{});
  }
  return acc;
}

// Gauss-Seidel stage on the slabs [s0, s1) of a sliced-ELL level: half wave
// per row, (blockIdx, threadIdx) -> row (s0 + hw / 64, hw % 64).  lim as in
// k_gs_sell (forward sweep from zero: entries of later stages skipped).  The
// row's r and diagonal are requested with its entries.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bgs_sell(const Slab* __restrict__ slabs, int s0, int s1,
                                                     const int* __restrict__ col, const T* __restrict__ val,
                                                     const T* __restrict__ diag, const T* __restrict__ r, T* x,
                                                     int lim) {
  const int hw = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) >> 5;
  const int s = s0 + (hw >> 6), i = hw & 63;
  if (s >= s1) return;
  // a lane past the slab's rows works on its last row and stores nothing
  // (no branch between the descriptor and the loads that need it)
  const Slab sl = load_slab(slabs, s);
  const int ii = min(i, sl.nrows - 1);
  const int c = threadIdx.x & 31;
  const int p = sl.row0 + ii;
  const T rp = r[(size_t)p * kNB + c];
  const T dp = diag[p];
  // the off-diagonal sum first, r added at the end, so that no wait for r
  // precedes the entry requests
  const T acc = half_row_sum<T, -1>(T(0), col + sl.off + ii, val + sl.off + ii, sl.width, c, x, lim);
  if (i < sl.nrows) x[(size_t)p * kNB + c] = (rp + acc) / dp;
}

// x = r / d on the rows p < rows0 (first stage of the forward sweep from zero)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bstage0_point(int rows0, const T* __restrict__ diag,
                                                          const T* __restrict__ r, T* __restrict__ x) {
  const int c = threadIdx.x & 31;
  for (int p = (blockIdx.x * kBlock + threadIdx.x) >> 5; p < rows0; p += gridDim.x * kRowsPerBlock)
    x[(size_t)p * kNB + c] = r[(size_t)p * kNB + c] / diag[p];
}

// MODE 0: s = r - A x;  MODE 1: s = A x with per-column x.s partials;
// MODE 2: s = A x.  Every block takes one contiguous run of the slabs' rows
// (kRowsPerBlock at a time), and the runs of an XCD's blocks are adjacent, so
// the rows an XCD handles at one time, and their neighbours, stay together.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_bresid_sell(const Slab* __restrict__ slabs, int nslabs,
                                                        const int* __restrict__ col, const T* __restrict__ val,
                                                        const T* __restrict__ diag, const T* __restrict__ r,
                                                        const T* __restrict__ x, T* __restrict__ s,
                                                        double* __restrict__ part) {
  const int c = threadIdx.x & 31;
  double dsum = 0.0;
  const int nhw = nslabs * 64;
  const int per = ((nhw + (int)gridDim.x - 1) / (int)gridDim.x + kRowsPerBlock - 1) / kRowsPerBlock * kRowsPerBlock;
  const int hw0 = xcd_block(blockIdx.x, gridDim.x) * per, hw1 = min(nhw, hw0 + per);
  for (int hw = hw0 + (int)(threadIdx.x >> 5); hw < hw1; hw += kRowsPerBlock) {
    const Slab sl = load_slab(slabs, hw >> 6);
    const int i = hw & 63;
    // past the slab's rows: its last row again, nothing stored
    const int ii = min(i, sl.nrows - 1);
    const int p = sl.row0 + ii;
    // the row's own values are requested with its entries
    const T xp = x[(size_t)p * kNB + c];
    const T dp = diag[p];
    const T rp = MODE == 0 ? r[(size_t)p * kNB + c] : T(0);
    const T acc = dp * xp + half_row_sum<T, 1>(T(0), col + sl.off + ii, val + sl.off + ii, sl.width, c, x, INT_MAX);
    if (i < sl.nrows) {
      if (MODE == 0) {
        s[(size_t)p * kNB + c] = rp - acc;
      } else {
        s[(size_t)p * kNB + c] = acc;
        if (MODE == 1) dsum += (double)xp * (double)acc;
      }
    }
  }
  if (MODE == 1) bcol_partials(dsum, 0, part);
}

// Off-group row sums of group g for column c: half wave h adds rows
// h, h + 2, ...; afterwards every lane holds a[q] for all rows q < k.
template <typename T, int KMAX>
__device__ __forceinline__ void bgroup_rowsums(int g, int h, int c, int k, const int* __restrict__ rec,
                                               const int* __restrict__ col, const T* __restrict__ val, const T* x,
                                               T (&a)[KMAX]) {
  constexpr int NT = (KMAX + 1) / 2;
  const int* gb = rec + (size_t)g * kRec + 3;
  T mine[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int l = 2 * t + h;
    T acc = T(0);
    if (l < k) {
      const int e1 = gb[l + 1];
      for (int e0 = gb[l]; e0 < e1; e0 += 4) {
        int cc[4];
        T vv[4], xx[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = min(e0 + u, e1 - 1);
          cc[u] = col[e];
          vv[u] = val[e];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) xx[u] = x[(size_t)cc[u] * kNB + c];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (e0 + u < e1) acc += vv[u] * xx[u];
      }
    }
    mine[t] = acc;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const T other = __shfl_xor(mine[t], 32, 64);
    a[2 * t] = h == 0 ? mine[t] : other;
    if (2 * t + 1 < KMAX) a[2 * t + 1] = h == 0 ? other : mine[t];
  }
}

// Gauss-Seidel stage on the groups [g0, g1): wave per group, every column
// relaxes the group's rows one after the other (forward or backward).
template <typename T, int KMAX>
__global__ __launch_bounds__(kBlock) void k_bgs_grp(int g0, int g1, const int* __restrict__ rec,
                                                    const int* __restrict__ col, const T* __restrict__ val,
                                                    const T* __restrict__ dblk, const T* __restrict__ r, T* x,
                                                    int backward) {
  const int g = __builtin_amdgcn_readfirstlane(g0 + xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) +
                                               (int)(threadIdx.x >> 6));
  if (g >= g1) return;
  const int lane = threadIdx.x & 63, h = lane >> 5, c = lane & 31;
  const int* R = rec + (size_t)g * kRec;
  const int p0 = R[0], k = R[1];
  const T* B = dblk + R[2];
  T xv[KMAX], rv[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    const size_t i = (size_t)(p0 + min(q, k - 1)) * kNB + c;
    const T xq = x[i], rq = r[i];
    xv[q] = (q < k) ? xq : T(0);
    rv[q] = (q < k) ? rq : T(0);
  }
  T a[KMAX];
  bgroup_rowsums<T, KMAX>(g, h, c, k, rec, col, val, x, a);
#pragma unroll
  for (int t = 0; t < KMAX; ++t) {
    const int ll = backward ? KMAX - 1 - t : t;
    if (ll < k) {
      T s = rv[ll] - a[ll];
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q < k && q != ll) s -= B[ll * k + q] * xv[q];
      xv[ll] = s / B[ll * k + ll];
    }
  }
#pragma unroll
  for (int q = 0; q < KMAX; ++q)
    if (q < k && (q & 1) == h) x[(size_t)(p0 + q) * kNB + c] = xv[q];
}

// ---- block per group, shared column lists
//
// On levels where every group's rows share one column list (rec[21] the row
// length, rec[20] the shift into gcol), one 256-thread block takes a group:
// its 8 half waves split the group's columns (half wave w: columns w, w + 8,
// ...), each column's block-vector row of x is gathered once and used for
// all k rows, and NU columns per half wave are in flight at a time.  The
// partial row sums go to LDS and the first wave adds them in half-wave order
// and finishes the group.  The record is read by the lanes (readlane for its
// fields); the first wave requests the group's own x, r and diagonal block
// before the column loop.
template <int KMAX>
constexpr int shared_nu() { return KMAX <= 2 ? 8 : KMAX == 4 ? 4 : 2; }

template <typename T, int KMAX>
struct SharedGroup {
  int p0, k, len, boff, cs, gb[KMAX];
};

template <typename T, int KMAX>
__device__ __forceinline__ SharedGroup<T, KMAX> shared_group(const int* __restrict__ rec, int g, int lane) {
  const int rw = rec[(size_t)g * kRec + min(lane, kRec - 1)];
  SharedGroup<T, KMAX> d;
  d.p0 = __builtin_amdgcn_readlane(rw, 0);
  d.k = __builtin_amdgcn_readlane(rw, 1);
  d.boff = __builtin_amdgcn_readlane(rw, 2);
  d.cs = __builtin_amdgcn_readlane(rw, 20);
#pragma unroll
  for (int q = 0; q < KMAX; ++q) d.gb[q] = __builtin_amdgcn_readlane(rw, 3 + q);
  d.len = __builtin_amdgcn_readlane(rw, 4) - d.gb[0];
  return d;
}

// This half wave's partial sums over its columns: acc[q] = sum of
// a_(row q, column j) x[column j] (column c of the block vector).
template <typename T, int KMAX>
__device__ __forceinline__ void shared_partial(const SharedGroup<T, KMAX>& d, int hw, int c,
                                               const int* __restrict__ gcol, const T* __restrict__ val, const T* x,
                                               T (&acc)[KMAX]) {
  constexpr int NU = shared_nu<KMAX>();
#pragma unroll
  for (int q = 0; q < KMAX; ++q) acc[q] = T(0);
  // rows past k read row 0's values (their sums are not used)
  int gq[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) gq[q] = (q < d.k) ? d.gb[q] : d.gb[0];
  for (int j0 = hw; j0 < d.len; j0 += 8 * NU) {
    int jj[NU], cc[NU];
    T vv[NU][KMAX], xx[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      jj[u] = min(j0 + 8 * u, d.len - 1);
      cc[u] = gcol[d.gb[0] + jj[u] + d.cs];
#pragma unroll
      for (int q = 0; q < KMAX; ++q) vv[u][q] = val[gq[q] + jj[u]];
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) xx[u] = x[(size_t)cc[u] * kNB + c];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const bool on = j0 + 8 * u < d.len;
#pragma unroll
      for (int q = 0; q < KMAX; ++q) acc[q] += (on ? vv[u][q] : T(0)) * xx[u];
    }
  }
}

// The first wave's group data: x and r of the rows for column c, and the
// diagonal block with lane t holding entry (t / KMAX, t % KMAX) (indices
// clamped into the group), for the block's LDS copy Bs.
template <typename T, int KMAX, bool WITH_R>
__device__ __forceinline__ void shared_own(const SharedGroup<T, KMAX>& d, int lane, int c,
                                           const T* __restrict__ dblk, const T* __restrict__ r, const T* x,
                                           T (&xv)[KMAX], T (&rv)[KMAX], T& bq) {
  const int tb = min(lane, KMAX * KMAX - 1);
  bq = dblk[d.boff + min(tb / KMAX, d.k - 1) * d.k + min(tb % KMAX, d.k - 1)];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    const size_t i = (size_t)(d.p0 + min(q, d.k - 1)) * kNB + c;
    xv[q] = x[i];
    rv[q] = WITH_R ? r[i] : T(0);
  }
}

// Gauss-Seidel stage on the groups [g0, g1), block per group (see above).
template <typename T, int KMAX>
__global__ __launch_bounds__(kBlock) void k_bgs_grps(int g0, int g1, const int* __restrict__ rec,
                                                     const int* __restrict__ gcol, const T* __restrict__ val,
                                                     const T* __restrict__ dblk, const T* __restrict__ r, T* x,
                                                     int backward) {
  __shared__ T part[8][KMAX][kNB];
  __shared__ T Bs[KMAX * KMAX];
  const int g = g0 + xcd_block(blockIdx.x, gridDim.x);
  if (g >= g1) return;
  const int lane = threadIdx.x & 63, hw = threadIdx.x >> 5, c = threadIdx.x & 31;
  const SharedGroup<T, KMAX> d = shared_group<T, KMAX>(rec, g, lane);
  T xv[KMAX], rv[KMAX], bq = T(0);
  if (threadIdx.x < 64) shared_own<T, KMAX, true>(d, lane, c, dblk, r, x, xv, rv, bq);
  T acc[KMAX];
  shared_partial<T, KMAX>(d, hw, c, gcol, val, x, acc);
#pragma unroll
  for (int q = 0; q < KMAX; ++q) part[hw][q][c] = acc[q];
  if (threadIdx.x < KMAX * KMAX) Bs[threadIdx.x] = bq;
  __syncthreads();
  if (threadIdx.x >= 64) return;
  const T(*B)[KMAX] = reinterpret_cast<const T(*)[KMAX]>(Bs);
  T a[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    T t = part[0][q][c];
#pragma unroll
    for (int w = 1; w < 8; ++w) t += part[w][q][c];
    a[q] = t;
    xv[q] = (q < d.k) ? xv[q] : T(0);
  }
#pragma unroll
  for (int t = 0; t < KMAX; ++t) {
    const int ll = backward ? KMAX - 1 - t : t;
    if (ll < d.k) {
      T s = rv[ll] - a[ll];
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q < d.k && q != ll) s -= B[ll][q] * xv[q];
      xv[ll] = s / B[ll][ll];
    }
  }
  if (lane < 32) {
#pragma unroll
    for (int q = 0; q < KMAX; ++q)
      if (q < d.k) x[(size_t)(d.p0 + q) * kNB + c] = xv[q];
  }
}

// s = r - A x on the groups [0, ng), block per group (see above).
template <typename T, int KMAX>
__global__ __launch_bounds__(kBlock) void k_bresid_grps(int ng, const int* __restrict__ rec,
                                                        const int* __restrict__ gcol, const T* __restrict__ val,
                                                        const T* __restrict__ dblk, const T* __restrict__ r,
                                                        const T* __restrict__ x, T* __restrict__ s) {
  __shared__ T part[8][KMAX][kNB];
  __shared__ T Bs[KMAX * KMAX];
  const int g = xcd_block(blockIdx.x, gridDim.x);
  if (g >= ng) return;
  const int lane = threadIdx.x & 63, hw = threadIdx.x >> 5, c = threadIdx.x & 31;
  const SharedGroup<T, KMAX> d = shared_group<T, KMAX>(rec, g, lane);
  T xv[KMAX], rv[KMAX], bq = T(0);
  if (threadIdx.x < 64) shared_own<T, KMAX, true>(d, lane, c, dblk, r, x, xv, rv, bq);
  T acc[KMAX];
  shared_partial<T, KMAX>(d, hw, c, gcol, val, x, acc);
#pragma unroll
  for (int q = 0; q < KMAX; ++q) part[hw][q][c] = acc[q];
  if (threadIdx.x < KMAX * KMAX) Bs[threadIdx.x] = bq;
  __syncthreads();
  if (threadIdx.x >= 32) return;
  const T(*B)[KMAX] = reinterpret_cast<const T(*)[KMAX]>(Bs);
#pragma unroll
  for (int l = 0; l < KMAX; ++l) {
    if (l < d.k) {
      T t = part[0][l][c];
#pragma unroll
      for (int w = 1; w < 8; ++w) t += part[w][l][c];
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q < d.k) t += B[l][q] * xv[q];
      s[(size_t)(d.p0 + l) * kNB + c] = rv[l] - t;
    }
  }
}

// forward sweep from x = 0 on a grouped level (thread per group and column)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bzero_stage0_grp(int ng, int ng0, const int* __restrict__ gstart,
                                                             const int* __restrict__ dboff,
                                                             const T* __restrict__ dblk, const T* __restrict__ r,
                                                             T* __restrict__ x) {
  const int c = threadIdx.x & 31;
  for (int g = (blockIdx.x * kBlock + threadIdx.x) >> 5; g < ng; g += gridDim.x * kRowsPerBlock) {
    const int p0 = gstart[g], k = gstart[g + 1] - p0;
    if (g >= ng0) {
      for (int q = 0; q < k; ++q) x[(size_t)(p0 + q) * kNB + c] = T(0);
      continue;
    }
    const T* B = dblk + dboff[g];
    T xv[kKmax];
#pragma unroll
    for (int l = 0; l < kKmax; ++l) {
      xv[l] = T(0);
      if (l < k) {
        T s = r[(size_t)(p0 + l) * kNB + c];
#pragma unroll
        for (int q = 0; q < kKmax; ++q)
          if (q < l) s -= B[l * k + q] * xv[q];
        xv[l] = s / B[l * k + l];
      }
    }
#pragma unroll
    for (int q = 0; q < kKmax; ++q)
      if (q < k) x[(size_t)(p0 + q) * kNB + c] = xv[q];
  }
}

// s = r - A x (MODE 0), s = A x with per-column x.s partials (MODE 1) or
// s = A x (MODE 2) on all groups; grid-stride, wave per group.
template <typename T, int KMAX, int MODE>
__global__ __launch_bounds__(kBlock) void k_bresid_grp(int ng, const int* __restrict__ rec,
                                                       const int* __restrict__ col, const T* __restrict__ val,
                                                       const T* __restrict__ dblk, const T* __restrict__ r,
                                                       const T* __restrict__ x, T* __restrict__ s,
                                                       double* __restrict__ part) {
  const int lane = threadIdx.x & 63, h = lane >> 5, c = lane & 31;
  double dsum = 0.0;
  const int gfirst = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) +
                                                    (int)(threadIdx.x >> 6));
  for (int g = gfirst; g < ng; g += gridDim.x * (kBlock / 64)) {
    const int* R = rec + (size_t)g * kRec;
    const int p0 = R[0], k = R[1];
    const T* B = dblk + R[2];
    T xv[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      const T xq = x[(size_t)(p0 + min(q, k - 1)) * kNB + c];
      xv[q] = (q < k) ? xq : T(0);
    }
    T a[KMAX];
    bgroup_rowsums<T, KMAX>(g, h, c, k, rec, col, val, x, a);
#pragma unroll
    for (int l = 0; l < KMAX; ++l) {
      if (l < k && (l & 1) == h) {
        T t = a[l];
#pragma unroll
        for (int q = 0; q < KMAX; ++q)
          if (q < k) t += B[l * k + q] * xv[q];
        const size_t i = (size_t)(p0 + l) * kNB + c;
        if (MODE == 0) {
          s[i] = r[i] - t;
        } else {
          s[i] = t;
          if (MODE == 1) dsum += (double)xv[l] * (double)t;
        }
      }
    }
  }
  if (MODE == 1) bcol_partials(dsum, 0, part);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bl1_init(int n, const T* __restrict__ dl1, const T* __restrict__ r,
                                                     T* __restrict__ x) {
  const int c = threadIdx.x & 31;
  for (int p = (blockIdx.x * kBlock + threadIdx.x) >> 5; p < n; p += gridDim.x * kRowsPerBlock)
    x[(size_t)p * kNB + c] = r[(size_t)p * kNB + c] / dl1[p];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bl1_update(int n, const T* __restrict__ dl1, const T* __restrict__ s,
                                                       T* __restrict__ x) {
  const int c = threadIdx.x & 31;
  for (int p = (blockIdx.x * kBlock + threadIdx.x) >> 5; p < n; p += gridDim.x * kRowsPerBlock)
    x[(size_t)p * kNB + c] += s[(size_t)p * kNB + c] / dl1[p];
}

// r_c = P^T s for block vectors: wave per aggregate, half wave h takes members
// h, h + 2, ... (four in flight), the halves are added with one exchange.
// Aggregate records, scut and INIT as in k_restrict (1: first Gauss-Seidel
// stage of the next level from x_c = 0, 2: first l1-Jacobi step); KMAX
// bounds the block widths k.  The record is read by the lanes and its fields
// taken with readlane; the diagonal block (INIT = 1), the member indices and
// their U entries are requested right after it, and the members' rows of s
// after the indices with no other wait: a member at or past scut (where
// s = 0) reads row scut - 1 instead and is weighted by zero.
template <typename T, int KMAX, int INIT>
__global__ __launch_bounds__(kBlock) void k_brestrict(int nagg, const int* __restrict__ arec,
                                                      const int* __restrict__ arows, const T* __restrict__ U,
                                                      const T* __restrict__ s, int scut, T* __restrict__ rc,
                                                      const T* __restrict__ cdblk, const T* __restrict__ cdl1,
                                                      T* __restrict__ xc) {
  const int a = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) +
                                               (int)(threadIdx.x >> 6));
  if (a >= nagg) return;
  const int lane = threadIdx.x & 63, h = lane >> 5, c = lane & 31;
  const int rw = arec[(size_t)a * kARec + min(lane, kARec - 1)];
  const int m0 = __builtin_amdgcn_readlane(rw, AR_M0), na = __builtin_amdgcn_readlane(rw, AR_NA);
  const int k = __builtin_amdgcn_readlane(rw, AR_K), c0 = __builtin_amdgcn_readlane(rw, AR_C0);
  const T* Ua = U + __builtin_amdgcn_readlane(rw, AR_UOFF);
  // lower triangle of the next level's diagonal block (INIT = 1; indices
  // clamped into the k x k block; without a block the level's first block,
  // at least k x k, is read and discarded)
  constexpr int NB = (INIT == 1) ? KMAX * (KMAX + 1) / 2 : 1;
  T bl[NB];
  int db = -1;
  if (INIT == 1) {
    db = __builtin_amdgcn_readlane(rw, AR_DB);
    const T* B = cdblk + max(db, 0);
#pragma unroll
    for (int l = 0; l < KMAX; ++l)
#pragma unroll
      for (int q = 0; q <= l; ++q) bl[l * (l + 1) / 2 + q] = B[min(l, k - 1) * k + min(q, k - 1)];
  }
  const int slast = max(scut - 1, 0);
  T acc[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) acc[q] = T(0);
  for (int l0 = h; l0 < na; l0 += 8) {
    int li[4], row[4];
    T sv[4], u[4][KMAX];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      li[v] = min(l0 + 2 * v, na - 1);
      row[v] = arows[m0 + li[v]];
#pragma unroll
      for (int q = 0; q < KMAX; ++q) u[v][q] = Ua[min(q, k - 1) * na + li[v]];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) sv[v] = s[(size_t)min(row[v], slast) * kNB + c];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T w = (l0 + 2 * v < na && row[v] < scut) ? sv[v] : T(0);
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q < k) acc[q] += u[v][q] * w;
    }
  }
#pragma unroll
  for (int q = 0; q < KMAX; ++q) acc[q] += __shfl_xor(acc[q], 32, 64);
#pragma unroll
  for (int q = 0; q < KMAX; ++q)
    if (q < k && (q & 1) == h) rc[(size_t)(c0 + q) * kNB + c] = acc[q];
  if (INIT == 1) {
    T xv[KMAX];
#pragma unroll
    for (int l = 0; l < KMAX; ++l) {
      T t = acc[l];
#pragma unroll
      for (int q = 0; q < l; ++q) t -= bl[l * (l + 1) / 2 + q] * xv[q];
      xv[l] = (db >= 0 && l < k) ? t / bl[l * (l + 1) / 2 + l] : T(0);
    }
#pragma unroll
    for (int q = 0; q < KMAX; ++q)
      if (q < k && (q & 1) == h) xc[(size_t)(c0 + q) * kNB + c] = xv[q];
  } else if (INIT == 2) {
#pragma unroll
    for (int q = 0; q < KMAX; ++q)
      if (q < k && (q & 1) == h) xc[(size_t)(c0 + q) * kNB + c] = acc[q] / cdl1[c0 + q];
  }
}

// x += P x_c for block vectors, in fine-row order (half wave per row), rows
// i < n, U entries at Urow[q * ld + i]
template <typename T, int KMAX>
__global__ __launch_bounds__(kBlock) void k_bprolong_rows(int n, int ld, const int* __restrict__ cinfo,
                                                          const T* __restrict__ Urow, const T* __restrict__ xc,
                                                          T* __restrict__ x) {
  const int c = threadIdx.x & 31;
  for (int i = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) >> 5; i < n; i += gridDim.x * kRowsPerBlock) {
    // as k_prolong_rows: every load requested together, entries past k zero
    const T xi = x[(size_t)i * kNB + c];
    const int ci = cinfo[i];
    T u[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) u[q] = Urow[(size_t)q * ld + i];
    const int c0 = ci >> 3, k = (ci & 7) + 1;
    T t = T(0);
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      const T v = xc[(size_t)(c0 + min(q, k - 1)) * kNB + c];
      t += (q < k ? u[q] : T(0)) * v;
    }
    x[(size_t)i * kNB + c] = xi + t;
  }
}

// Z = A R for the coarsest level: A dense row-major with leading dimension ld
// (a multiple of 64, entries past n zero, rows up to ld readable), R and Z
// n x 32.  A block computes 8 * RPH rows: half wave hw holds rows
// blk * 8 * RPH + hw + 8 t (t < RPH) for column c; R is staged through LDS in
// chunks of 64 rows and every A entry is read once per block.
template <int RPH>
__global__ __launch_bounds__(kBlock) void k_bgemm(int n, int ld, const double* __restrict__ A,
                                                  const double* __restrict__ R, double* __restrict__ Z) {
  __shared__ double Rs[64][kNB];
  const int c = threadIdx.x & 31, hw = threadIdx.x >> 5;
  const int row0 = blockIdx.x * 8 * RPH + hw;
  double acc[RPH];
  const double* Ar[RPH];
#pragma unroll
  for (int t = 0; t < RPH; ++t) {
    acc[t] = 0.0;
    Ar[t] = A + (size_t)min(row0 + 8 * t, ld - 1) * ld;
  }
  for (int k0 = 0; k0 < ld; k0 += 64) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + kBlock * u;
      const int kr = e >> 5, cc = e & 31;
      Rs[kr][cc] = (k0 + kr < n) ? R[(size_t)(k0 + kr) * kNB + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 64; kk += 4) {
      const double r0 = Rs[kk][c], r1 = Rs[kk + 1][c], r2 = Rs[kk + 2][c], r3 = Rs[kk + 3][c];
#pragma unroll
      for (int t = 0; t < RPH; ++t) {
        const double2 a01 = *reinterpret_cast<const double2*>(Ar[t] + k0 + kk);
        const double2 a23 = *reinterpret_cast<const double2*>(Ar[t] + k0 + kk + 2);
        acc[t] += a01.x * r0 + a01.y * r1 + a23.x * r2 + a23.y * r3;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < RPH; ++t) {
    const int i = row0 + 8 * t;
    if (i < n) Z[(size_t)i * kNB + c] = acc[t];
  }
}

typedef double dbl4_t __attribute__((ext_vector_type(4)));

// Z = A R for the coarsest level on matrix cores (binary64 16x16x4 MFMA).
// Block (row tile t, split ks) owns rows 16 t .. 16 t + 15 and all 32
// columns for the KS-th share ks of the inner dimension; its W waves split
// that share again in contiguous ranges and add their 16 x 32 partial tiles
// in LDS in wave order.  With KS = 1 the tile goes to Z, else to
// P + ks * n * 32 and k_bsum_splits adds the splits in order (deterministic).
// Per 16-wide inner step lane l holds A[16 t + l % 16][k + 4 (l / 16) .. + 3]
// (one 32-byte load); MFMA j of the step multiplies the entries j of those
// quads with the matching rows of R, so the inner index is permuted the same
// way on both operands.  Accumulator entry i of lane l is D[4 i + l / 16][l % 16].
template <int W>
__global__ __launch_bounds__(64 * W) void k_bgemm_mfma(int n, int ld, const double* __restrict__ A,
                                                       const double* __restrict__ R, double* __restrict__ Z) {
  __shared__ double part[W][16][kNB];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int r0 = blockIdx.x * 16, ks = blockIdx.y, KS = gridDim.y;
  const int nk = ld / 16;
  const int s0 = ((ks * W + w) * nk) / (KS * W), s1 = ((ks * W + w + 1) * nk) / (KS * W);
  const double* Arow = A + (size_t)(r0 + li) * ld + 4 * lq;
  dbl4_t acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int s = s0; s < s1; ++s) {
    const int kq = 16 * s + 4 * lq;
    const double2 a01 = *reinterpret_cast<const double2*>(Arow + 16 * s);
    const double2 a23 = *reinterpret_cast<const double2*>(Arow + 16 * s + 2);
    double b0[4], b1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kr = kq + j;
      const bool in = kr < n;
      const size_t o = (size_t)(in ? kr : 0) * kNB + li;
      b0[j] = in ? R[o] : 0.0;
      b1[j] = in ? R[o + 16] : 0.0;
    }
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a01.x, b0[0], acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a01.x, b1[0], acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a01.y, b0[1], acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a01.y, b1[1], acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a23.x, b0[2], acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a23.x, b1[2], acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a23.y, b0[3], acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a23.y, b1[3], acc1, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    part[w][4 * i + lq][li] = acc0[i];
    part[w][4 * i + lq][16 + li] = acc1[i];
  }
  __syncthreads();
  double* out = Z + (size_t)ks * n * kNB;
  for (int e = threadIdx.x; e < 16 * kNB; e += 64 * W) {
    const int row = e / kNB, c = e % kNB;
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < W; ++q) sum += part[q][row][c];
    if (r0 + row < n) out[(size_t)(r0 + row) * kNB + c] = sum;
  }
}

// Z[e] = sum over ks = 0 .. KS-1 of P[ks * m + e], in that order
__global__ __launch_bounds__(kBlock) void k_bsum_splits(int m, int KS, const double* __restrict__ P,
                                                        double* __restrict__ Z) {
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < m; e += gridDim.x * kBlock) {
    double s = P[e];
    for (int ks = 1; ks < KS; ++ks) s += P[(size_t)ks * m + e];
    Z[e] = s;
  }
}

// -------------------------------------------- independent problems (batch)

// y = blockdiag(A_p) x on the coarsest level of a batch: wave per row; the
// rows [coff[p], coff[p+1]) belong to problem p, whose inverse is dense
// row-major with leading dimension cnp[p] (even) at A + aoff[p].
__global__ __launch_bounds__(kBlock) void k_gemv_batch(int n, const int* __restrict__ cprob,
                                                       const int* __restrict__ coff, const int* __restrict__ cnp,
                                                       const int64_t* __restrict__ aoff,
                                                       const double* __restrict__ A, const double* __restrict__ x,
                                                       double* __restrict__ y) {
  const int i = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (i >= n) return;
  const int lane = threadIdx.x & 63;
  const int p = cprob[i], c0 = coff[p], m = coff[p + 1] - c0, ld = cnp[p];
  const double2* Ai = reinterpret_cast<const double2*>(A + aoff[p] + (size_t)(i - c0) * ld);
  const double* xp = x + c0;
  double a0 = 0.0, a1 = 0.0;
  const int m2 = m / 2;
  int j = lane;
  for (; j + 64 < m2; j += 128) {
    const double2 v0 = Ai[j], v1 = Ai[j + 64];
    a0 += v0.x * xp[2 * j] + v0.y * xp[2 * j + 1];
    a1 += v1.x * xp[2 * j + 128] + v1.y * xp[2 * j + 129];
  }
  for (; j < m2; j += 64) {
    const double2 v = Ai[j];
    a0 += v.x * xp[2 * j] + v.y * xp[2 * j + 1];
  }
  if ((m & 1) && lane == 0) a1 += A[aoff[p] + (size_t)(i - c0) * ld + m - 1] * xp[m - 1];
  const double acc = wave_sum(a0 + a1);
  if (lane == 0) y[i] = acc;
}

// Problem p owns the entries idx[j], j in [poff[p], poff[p+1]), of the level-0
// vectors.  Grid (chunks, problems); partials at part[(v * nprob + p) *
// gridDim.x + chunk].  With act given, the blocks of a stopped problem
// (act[p * S_NSCAL] == 0) write zero partials and touch nothing else.
__device__ __forceinline__ bool pstopped(const double* act, int p) {
  return act != nullptr && act[(size_t)p * S_NSCAL] == 0.0;
}

template <int NV>
__global__ __launch_bounds__(kBlock) void k_pdot(const int* __restrict__ poff, const int* __restrict__ idx,
                                                 const double* __restrict__ a, const double* __restrict__ b,
                                                 const double* __restrict__ c, const double* __restrict__ d,
                                                 double* __restrict__ part, const double* __restrict__ act) {
  __shared__ double lds[4];
  const int p = blockIdx.y, j1 = poff[p + 1];
  if (pstopped(act, p)) {
    if (threadIdx.x == 0) {
      part[(size_t)p * gridDim.x + blockIdx.x] = 0.0;
      if (NV > 1) part[(size_t)(gridDim.y + p) * gridDim.x + blockIdx.x] = 0.0;
    }
    return;
  }
  double s0 = 0.0, s1 = 0.0;
  for (int j = poff[p] + blockIdx.x * kBlock + threadIdx.x; j < j1; j += gridDim.x * kBlock) {
    const int i = idx[j];
    s0 += a[i] * b[i];
    if (NV > 1) s1 += c[i] * d[i];
  }
  s0 = block_sum(s0, lds);
  if (NV > 1) s1 = block_sum(s1, lds);
  if (threadIdx.x == 0) {
    part[(size_t)p * gridDim.x + blockIdx.x] = s0;
    if (NV > 1) part[(size_t)(gridDim.y + p) * gridDim.x + blockIdx.x] = s1;
  }
}

__global__ __launch_bounds__(kBlock) void k_paxpy2_dot(const int* __restrict__ poff, const int* __restrict__ idx,
                                                       const double* __restrict__ scal, const double* __restrict__ pv,
                                                       const double* __restrict__ q, double* __restrict__ x,
                                                       double* __restrict__ r, double* __restrict__ part, int skip) {
  __shared__ double lds[4];
  const int p = blockIdx.y, j1 = poff[p + 1];
  const double alpha = scal[p * S_NSCAL + S_ALPHA];
  const bool act = scal[p * S_NSCAL + S_ACT] != 0.0;
  if (skip && !act) {
    if (threadIdx.x == 0) part[(size_t)p * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
  double s = 0.0;
  for (int j = poff[p] + blockIdx.x * kBlock + threadIdx.x; j < j1; j += gridDim.x * kBlock) {
    const int i = idx[j];
    double ri = r[i];
    if (act) {
      x[i] += alpha * pv[i];
      ri -= alpha * q[i];
      r[i] = ri;
    }
    s += ri * ri;
  }
  s = block_sum(s, lds);
  if (threadIdx.x == 0) part[(size_t)p * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_pxpay(const int* __restrict__ poff, const int* __restrict__ idx,
                                                  const double* __restrict__ scal, const double* __restrict__ z,
                                                  double* __restrict__ pv, int skip) {
  const int p = blockIdx.y, j1 = poff[p + 1];
  if (skip && scal[p * S_NSCAL + S_ACT] == 0.0) return;
  const double beta = scal[p * S_NSCAL + S_BETA];
  for (int j = poff[p] + blockIdx.x * kBlock + threadIdx.x; j < j1; j += gridDim.x * kBlock) {
    const int i = idx[j];
    pv[i] = z[i] + beta * pv[i];
  }
}

}  // namespace mvamg
