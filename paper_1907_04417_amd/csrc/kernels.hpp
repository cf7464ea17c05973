// Device kernels of the solve phase (gfx950, 64-lane wavefronts).
//
// Storage of a level (rows renumbered into smoother order, so that every
// smoother stage is a contiguous row range and every group a contiguous run):
//   * point levels with short rows: sliced ELL, 64-row slabs, entries of a
//     slab column-major (lane i reads row i's j-th entry at off + 64 j + i,
//     one coalesced 512-byte load per wave for binary64 values);
//   * other levels: CSR of the entries outside the diagonal blocks, G lanes
//     per group striding over the group's contiguous entry range;
//   * the k x k diagonal block of every group, dense row-major.
// All kernels are HBM-bandwidth bound (about 2 flops per 12 bytes), so they
// use plain vector FMA, not matrix cores.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>

#include "hier_host.hpp"

namespace mvamg {

constexpr int kBlock = 256;

// Logical block index with consecutive logical blocks on one XCD.  Blocks are
// handed to the 8 XCDs round robin (block b to XCD b % 8) and each XCD has
// its own L2.  Rows that share neighbours (or, in a transfer, the residual
// lines of neighbouring aggregates) sit in nearby blocks; handed out round
// robin they are fetched once per XCD, unless XCD x works on one contiguous
// run of logical blocks.  A bijection of [0, nb) for any nb.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
  return x * q + min(x, r) + i;
}

// ----------------------------------------------------------- reductions

enum Scalar {
  S_RHO = 0,   // r.z of the current iterate
  S_PQ = 1,    // p.A p
  S_ALPHA = 2, // rho / pq
  S_RR = 3,    // r.r
  S_BETA = 4,  // CG beta
  S_FLAG = 5,  // breakdown flag (p.Ap <= 0)
  S_R0 = 6,    // ||r_0||^2
  S_ZQ = 7,    // z.q (flexible beta)
  S_STEPS = 15,  // CG steps finished in this solve (their scalars alternate between two host slots)
  S_NSCAL = 16
};

enum RedMode { M_STORE_RR = 0, M_PQ = 1, M_RHO0 = 2, M_RZ = 3, M_RZ_FLEX = 4, M_STORE_R0 = 5, M_NONE = 6 };

// Batches of independent problems: a work unit (slab, row, aggregate) of
// problem q is skipped when act is given and act[q * S_NSCAL] == 0 (the
// problem has stopped; act points at its per-problem S_ACT flag).
struct Skip {
  const int* uprob;   // problem of each work unit
  const double* act;  // nullptr: nothing is skipped
};

__device__ __forceinline__ bool skipped(const Skip& k, int unit) {
  return k.act != nullptr && k.act[(size_t)k.uprob[unit] * S_NSCAL] == 0.0;
}

struct Red {
  double* part;  // one slot per block and value (2 * grid)
};

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_value(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Sum of v over aligned groups of min(LPR, 16) lanes (quad_perm [1,0,3,2],
// quad_perm [2,3,0,1], row_half_mirror, row_mirror); every lane of the group
// holds the result.
template <int LPR, typename T>
__device__ __forceinline__ T lanes_sum(T v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  if (LPR >= 16) v += dpp_mov<0x140>(v);
  return v;
}

// Sum over the 64 lanes (DPP inside each 16-lane row, then the four row sums
// in order); every lane holds the result.
__device__ __forceinline__ double wave_sum(double v) {
  v = lanes_sum<16>(v);
  return ((lane_value(v, 0) + lane_value(v, 16)) + lane_value(v, 32)) + lane_value(v, 48);
}

template <int G>
__device__ __forceinline__ double seg_sum(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

template <int G>
__device__ __forceinline__ float seg_sum(float v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// Sum over a 256-thread block in a fixed order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = ((lds[0] + lds[1]) + lds[2]) + lds[3];
  __syncthreads();
  return t;
}

// rho and alpha are read by the caller before the sums (their loads overlap
// with the partial loads).
__device__ __forceinline__ void epilogue(int mode, double v0, double v1, double rho, double alpha, double* scal) {
  switch (mode) {
    case M_STORE_RR: scal[S_RR] = v0; break;
    case M_STORE_R0: scal[S_R0] = v0; break;
    case M_PQ:
      scal[S_PQ] = v0;
      if (!(v0 > 0.0)) scal[S_FLAG] = 1.0;
      scal[S_ALPHA] = rho / v0;
      break;
    case M_RHO0: scal[S_RHO] = v0; break;
    case M_RZ:
      scal[S_BETA] = v0 / rho;
      scal[S_RHO] = v0;
      break;
    case M_RZ_FLEX:
      scal[S_ZQ] = v1;
      scal[S_BETA] = -alpha * v1 / rho;
      scal[S_RHO] = v0;
      break;
  }
}

// Block partial sums of up to two values: part[b] and part[grid + b].  A
// one-block finisher (k_finish) adds the partials in block order and applies
// the epilogue, so results are deterministic and need no inter-block
// synchronisation inside a kernel.
template <int NV>
__device__ __forceinline__ void block_partials(double a0, double a1, double* part) {
  __shared__ double lds[4];
  const double b0 = block_sum(a0, lds);
  double b1 = 0.0;
  if (NV > 1) b1 = block_sum(a1, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = b0;
    if (NV > 1) part[gridDim.x + blockIdx.x] = b1;
  }
}

// The finisher: one block of kFinish threads; thread t adds the partials
// t + kFinish u in u order, eight loads in flight, then the wave sums are
// added in wave order.  host (optional): mapped host memory that also gets
// the scalars (system-scope stores; the host reads them after the stream).
constexpr int kFinish = 1024;
template <int NV>
__global__ __launch_bounds__(kFinish) void k_finish(int nparts, const double* __restrict__ part, double* scal,
                                                    int mode, double* host) {
  __shared__ double lds[2][kFinish / 64];
  const double rho = scal[S_RHO], alpha = scal[S_ALPHA];
  double s0 = 0.0, s1 = 0.0;
  for (int i0 = threadIdx.x; i0 < nparts; i0 += 8 * kFinish) {
    double v0[8], v1[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * kFinish;
      v0[u] = (i < nparts) ? part[i] : 0.0;
      v1[u] = (NV > 1 && i < nparts) ? part[nparts + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      s0 += v0[u];
      s1 += v1[u];
    }
  }
  s0 = wave_sum(s0);
  if (NV > 1) s1 = wave_sum(s1);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    lds[0][w] = s0;
    lds[1][w] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0.0, t1 = 0.0;
    for (int q = 0; q < kFinish / 64; ++q) {
      t0 += lds[0][q];
      t1 += lds[1][q];
    }
    epilogue(mode, t0, t1, rho, alpha, scal);
    if (host != nullptr) {
      // step g of the solve (g = scal[S_STEPS]) writes host slot g mod 2, so
      // the host can still read step g while step g + 1 runs
      double v[S_NSCAL];
#pragma unroll
      for (int i = 0; i < S_NSCAL; ++i) v[i] = scal[i];
      double* slot = host + ((int)v[S_STEPS] & 1) * S_NSCAL;
      scal[S_STEPS] = v[S_STEPS] + 1.0;
#pragma unroll
      for (int i = 0; i < S_NSCAL; ++i) __hip_atomic_store(slot + i, v[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// ------------------------------------------- K-cycle inner iterations
//
// Two flexible-CG iterations on a coarse level (the K-cycle's coarse
// correction): NV inner products as block partials, one block adding them in
// block order, and the two vector updates that read the results.  Scalars of
// level m live at ks[0..4]: c1.v1, c1.g, then c2.v1, c2.v2, c2.r2.

template <int NV>
__global__ __launch_bounds__(kBlock) void k_kdots(int n, const double* __restrict__ a0, const double* __restrict__ b0,
                                                  const double* __restrict__ a1, const double* __restrict__ b1,
                                                  const double* __restrict__ a2, const double* __restrict__ b2,
                                                  double* __restrict__ part) {
  __shared__ double lds[4];
  double s[3] = {0.0, 0.0, 0.0};
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) {
    s[0] += a0[p] * b0[p];
    if (NV > 1) s[1] += a1[p] * b1[p];
    if (NV > 2) s[2] += a2[p] * b2[p];
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double t = block_sum(s[k], lds);
    if (threadIdx.x == 0) part[k * gridDim.x + blockIdx.x] = t;
  }
}

// out[k] = sum of the nparts partials of value k, added in block order.
template <int NV>
__global__ __launch_bounds__(kBlock) void k_kfinish(int nparts, const double* __restrict__ part,
                                                    double* __restrict__ out) {
  __shared__ double lds[4];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kBlock) s += part[k * nparts + i];
    const double t = block_sum(s, lds);
    if (threadIdx.x == 0) out[k] = t;
  }
}

// r2 = g - alpha1 v1, alpha1 = (c1.g) / (c1.v1)
__global__ __launch_bounds__(kBlock) void k_kresid(int n, const double* __restrict__ ks, const double* __restrict__ g,
                                                   const double* __restrict__ v1, double* __restrict__ r2) {
  const double alpha1 = ks[1] / ks[0];
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) r2[p] = g[p] - alpha1 * v1[p];
}

// y = alpha1 c1 + alpha2 (c2 - (gamma / rho1) c1): the second direction made
// A-orthogonal to the first; beta = p2^T A p2 = c2.v2 - gamma^2 / rho1,
// alpha2 = (c2.r2) / beta.  y may alias c1.
__global__ __launch_bounds__(kBlock) void k_kcombine(int n, const double* __restrict__ ks, const double* c1,
                                                     const double* __restrict__ c2, double* y) {
  const double rho1 = ks[0], alpha1 = ks[1] / rho1, gamma = ks[2];
  const double beta = ks[3] - gamma * gamma / rho1, alpha2 = ks[4] / beta;
  const double t1 = alpha1 - alpha2 * gamma / rho1;
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) y[p] = t1 * c1[p] + alpha2 * c2[p];
}

// ------------------------------------------------------- vector kernels

// out = a x + b y (out may alias x or y)
__global__ __launch_bounds__(kBlock) void k_axpby(int n, double a, const double* x, double b, const double* y,
                                                  double* out) {
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) out[p] = a * x[p] + b * y[p];
}

// x = x / d
__global__ __launch_bounds__(kBlock) void k_div(int n, double d, double* __restrict__ x) {
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) x[p] = x[p] / d;
}

// out[p] = in[map[perm[p]]] and its inverse: a batch's part in its own
// numbering, read from and written to the caller's rows
__global__ __launch_bounds__(kBlock) void k_gather2(int n, const int* __restrict__ perm, const int* __restrict__ map,
                                                    const double* __restrict__ in, double* __restrict__ out) {
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) out[p] = in[map[perm[p]]];
}
__global__ __launch_bounds__(kBlock) void k_scatter2(int n, const int* __restrict__ perm, const int* __restrict__ map,
                                                     const double* __restrict__ in, double* __restrict__ out) {
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) out[map[perm[p]]] = in[p];
}

// out[perm[p]] += s in[p] (perm a permutation: no two threads write one entry)
__global__ __launch_bounds__(kBlock) void k_scatter_axpy(int n, const int* __restrict__ perm, double s,
                                                         const double* __restrict__ in, double* __restrict__ out) {
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) out[perm[p]] += s * in[p];
}

__global__ __launch_bounds__(kBlock) void k_gather(int n, const int* __restrict__ perm,
                                                   const double* __restrict__ in, double* __restrict__ out) {
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) out[p] = in[perm[p]];
}

__global__ __launch_bounds__(kBlock) void k_scatter(int n, const int* __restrict__ perm,
                                                    const double* __restrict__ in, double* __restrict__ out) {
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) out[perm[p]] = in[p];
}

template <typename Ti, typename To>
__global__ __launch_bounds__(kBlock) void k_cast(int n, const Ti* __restrict__ in, To* __restrict__ out) {
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) out[p] = (To)in[p];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, T v, T* __restrict__ out) {
  for (int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x; p < n; p += (int64_t)gridDim.x * kBlock) out[p] = v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(int n, const T* __restrict__ in, T* __restrict__ out) {
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) out[p] = in[p];
}

// sum of a.b (and c.d) with an epilogue
template <int NV>
__global__ __launch_bounds__(kBlock) void k_dot(int n, const double* __restrict__ a, const double* __restrict__ b,
                                                const double* __restrict__ c, const double* __restrict__ d, Red red) {
  double s0 = 0.0, s1 = 0.0;
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) {
    s0 += a[p] * b[p];
    if (NV > 1) s1 += c[p] * d[p];
  }
  block_partials<NV>(s0, s1, red.part);
}


// x += alpha p (the previous step's, deferred to here: p is read anyway),
// then p = z + beta p
__global__ __launch_bounds__(kBlock) void k_xpay(int n, const double* __restrict__ scal, const double* __restrict__ z,
                                                 double* __restrict__ p, double* __restrict__ x) {
  const double beta = scal[S_BETA], alpha = scal[S_ALPHA];
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double pi = p[i];
    x[i] += alpha * pi;
    p[i] = z[i] + beta * pi;
  }
}

// x += alpha p: the deferred update of the last CG step
__global__ __launch_bounds__(kBlock) void k_x_update(int n, const double* __restrict__ scal,
                                                     const double* __restrict__ p, double* __restrict__ x) {
  const double alpha = scal[S_ALPHA];
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) x[i] += alpha * p[i];
}

// ------------------------------------------------- sliced-ELL (point) levels

// Column indices of the slabs: 32-bit (col), or, where a slab's j-th entries
// span at most 65535 columns, 16-bit deltas col16 from a per-(slab, entry
// position) base cbase[scb[s] + j] (scb[s] = -1: 32-bit; the bases of a slab
// are padded to a multiple of 8 with the last one).  col16 (and the value
// codes) are lane-packed: the eight slots j0 .. j0 + 7 of a lane are adjacent
// at pk[s] + 64 j0 + 8 lane, one 16-byte load; slots past the width point at
// a row and their products are dropped.
struct SellCols {
  const int* __restrict__ col;
  const uint16_t* __restrict__ col16;
  const int* __restrict__ cbase;
  const int* __restrict__ scb;
  const int* __restrict__ pk;
};

// Columns of the entries j0 .. j0 + 7 (clamped to the slab's width, or
// packed slots past it) of slab row `lane`; cb = scb[slab], po = pk[slab]
// (wave-uniform).
__device__ __forceinline__ void sell_cols8(const SellCols& C, const Slab& sl, int cb, int po, int lane, int j0,
                                           int cc[8]) {
  if (cb >= 0) {
    const uint4 w = *reinterpret_cast<const uint4*>(C.col16 + po + 64 * j0 + 8 * lane);
    const int* b = C.cbase + cb + j0;
    const unsigned d[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int u = 0; u < 8; ++u) cc[u] = b[u] + (int)((d[u >> 1] >> (16 * (u & 1))) & 0xffffu);
  } else {
    const int* c = C.col + sl.off + lane;
#pragma unroll
    for (int u = 0; u < 8; ++u) cc[u] = c[64 * min(j0 + u, sl.width - 1)];
  }
}

// Values of a sliced-ELL level: the entries (slab layout, as the columns)
// and the diagonal, each either stored or as 1-byte codes into a table of at
// most 256 values (the same binary64 values, or their binary32 roundings).
// A kernel stages the tables in LDS (stage_tables) and looks codes up there.
template <typename T>
struct SellVals {
  const T* __restrict__ val;
  const T* __restrict__ diag;
  const uint8_t* __restrict__ vcode;  // nullptr: read val
  const uint8_t* __restrict__ dcode;  // nullptr: read diag
  const T* __restrict__ vtab;
  const T* __restrict__ dtab;
  int nvtab, ndtab;
};

constexpr int kTab = 256;

// All threads of the block; ends with a barrier.  Thread t requests entry t
// of both tables before writing either (one round trip).
template <typename T>
__device__ __forceinline__ void stage_tables(const SellVals<T>& V, T* vt, T* dt) {
  static_assert(kBlock >= kTab, "one table entry per thread");
  const int t = threadIdx.x;
  T a = T(0), b = T(0);
  if (V.vcode) a = V.vtab[min(t, V.nvtab - 1)];
  if (V.dcode) b = V.dtab[min(t, V.ndtab - 1)];
  if (V.vcode && t < V.nvtab) vt[t] = a;
  if (V.dcode && t < V.ndtab) dt[t] = b;
  __syncthreads();
}

// A slab descriptor in one 16-byte load.
__device__ __forceinline__ Slab load_slab(const Slab* __restrict__ slabs, int s) {
  const int4 v = *reinterpret_cast<const int4*>(slabs + s);
  return Slab{v.x, v.y, v.z, v.w};
}

// Values of the entries j0 .. j0 + 7 (clamped to the slab's width, or
// packed slots past it) of slab row `lane`; po = pk[slab].
template <typename T>
__device__ __forceinline__ void sell_vals8(const SellVals<T>& V, const T* vt, const Slab& sl, int po, int lane,
                                           int j0, T vv[8]) {
  if (V.vcode) {
    const uint2 w = *reinterpret_cast<const uint2*>(V.vcode + po + 64 * j0 + 8 * lane);
#pragma unroll
    for (int u = 0; u < 8; ++u) vv[u] = vt[((u < 4 ? w.x : w.y) >> (8 * (u & 3))) & 0xffu];
  } else {
    const T* v = V.val + sl.off + lane;
#pragma unroll
    for (int u = 0; u < 8; ++u) vv[u] = v[64 * min(j0 + u, sl.width - 1)];
  }
}

template <typename T>
__device__ __forceinline__ T sell_diag(const SellVals<T>& V, const T* dt, int p) {
  return V.dcode ? dt[V.dcode[p]] : V.diag[p];
}

// One Gauss-Seidel stage: x_p <- (r_p - sum_{j != p} a_pj x_j) / a_pp for the
// rows of the slabs [s0, s1) (rows of one stage are not coupled).  In the
// forward sweep from x = 0, lim is the stage's first row: entries of later
// stages (column >= lim) multiply values that are still zero and are
// skipped, so those rows need not be cleared beforehand; otherwise lim is
// past every row.  DOT = 1 (binary64, no batch skipping): the block also
// writes the sum of x_p r_p over its new rows to part[blockIdx.x] (the last
// sweep of a cycle then yields the partials of z.r).
//
// Load order: the slab's descriptors with the value tables, then (after the
// tables' barrier) r, the diagonal and the entries together, then the
// neighbour values.  A lane past its slab's rows works on the slab's last
// row and stores nothing, and a skipped entry is a zero weight, so no branch
// puts a wait between these requests.
template <typename T, int DOT>
__global__ __launch_bounds__(kBlock) void k_gs_sell(const Slab* __restrict__ slabs, int s0, int s1,
                                                    SellCols C, SellVals<T> V, const T* __restrict__ r, T* x,
                                                    Skip sk, int lim, double* __restrict__ part) {
  __shared__ T vt[kTab], dt[kTab];
  const int s = s0 + xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int sc = min(s, s1 - 1);
  const Slab sl = load_slab(slabs, sc);
  const int cb = C.scb[sc], po = C.pk[sc];
  // (wave-uniform; a batch's stopped problems skip all further loads)
  const bool act = s < s1 && !skipped(sk, sc);
  stage_tables(V, vt, dt);
  double dsum = 0.0;
  if (act) {
    const int li = min(lane, sl.nrows - 1);
    const int p = sl.row0 + li;
    const T rp = r[p];
    const int dcode = V.dcode ? (int)V.dcode[p] : 0;
    const T dval = V.dcode ? T(0) : V.diag[p];
    T acc = rp;
    // entries in batches of 8: all index and value loads, then all gathers, then the sums
    for (int j0 = 0; j0 < sl.width; j0 += 8) {
      int cc[8];
      T vv[8], xx[8];
      sell_cols8(C, sl, cb, po, li, j0, cc);
      sell_vals8(V, vt, sl, po, li, j0, vv);
#pragma unroll
      for (int u = 0; u < 8; ++u) xx[u] = x[min(cc[u], lim - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const T w = (j0 + u < sl.width && cc[u] < lim) ? vv[u] : T(0);
        acc -= w * xx[u];
      }
    }
    const T xn = acc / (V.dcode ? dt[dcode] : dval);
    if (lane < sl.nrows) {
      x[p] = xn;
      if (DOT) dsum = (double)xn * (double)rp;
    }
  }
  if (DOT) block_partials<1>(dsum, 0.0, part);
}

// r -= alpha q; sum r.r (x += alpha p follows in k_xpay or k_x_update).
// rows0 > 0: also the first stage of the next cycle's forward sweep from
// zero on a point fine level, z_p = r_p / a_pp for p < rows0 (as
// k_stage0_point, from the new r).
__global__ __launch_bounds__(kBlock) void k_axpy_dot(int n, const double* __restrict__ scal,
                                                     const double* __restrict__ q, double* __restrict__ r, Red red,
                                                     int rows0, SellVals<double> V, double* __restrict__ z) {
  __shared__ double vt[1], dt[kTab];
  V.vcode = nullptr;  // entries are not read
  if (rows0 > 0) stage_tables(V, vt, dt);
  const double alpha = scal[S_ALPHA];
  double s = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    s += ri * ri;
    if (i < rows0) z[i] = ri / sell_diag(V, dt, i);
  }
  block_partials<1>(s, 0.0, red.part);
}

// First stage of the forward sweep from x = 0 on a point level: x_p = r_p /
// a_pp for the rows p < rows0 (the other rows are written by their stages).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_stage0_point(int rows0, SellVals<T> V, const T* __restrict__ r,
                                                         T* __restrict__ x, Skip sk) {
  __shared__ T vt[1], dt[kTab];
  V.vcode = nullptr;  // entries are not read
  stage_tables(V, vt, dt);
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < rows0; p += gridDim.x * kBlock)
    if (!skipped(sk, p)) x[p] = r[p] / sell_diag(V, dt, p);
}

// s = r - A x (MODE 0), y = A x with sum x.y (MODE 1, binary64 only), or y = A x
// (MODE 2).  Load order and clamping as in k_gs_sell; the diagonal term is
// added after the off-diagonal sum.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_resid_sell(const Slab* __restrict__ slabs, int nslabs,
                                                       SellCols C, SellVals<T> V, const T* __restrict__ r,
                                                       const T* __restrict__ x, T* __restrict__ s, Red red, Skip sk) {
  __shared__ T vt[kTab], dt[kTab];
  const int sidx = xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int sc = min(sidx, nslabs - 1);
  const Slab sl = load_slab(slabs, sc);
  const int cb = C.scb[sc], po = C.pk[sc];
  // (wave-uniform; a batch's stopped problems skip all further loads)
  const bool act = sidx < nslabs && !skipped(sk, sc);
  stage_tables(V, vt, dt);
  double dsum = 0.0;
  if (act) {
    const int li = min(lane, sl.nrows - 1);
    const int p = sl.row0 + li;
    const T xp = x[p];
    const T rp = MODE == 0 ? r[p] : T(0);
    const int dcode = V.dcode ? (int)V.dcode[p] : 0;
    const T dval = V.dcode ? T(0) : V.diag[p];
    T acc = T(0);
    for (int j0 = 0; j0 < sl.width; j0 += 8) {
      int cc[8];
      T vv[8], xx[8];
      sell_cols8(C, sl, cb, po, li, j0, cc);
      sell_vals8(V, vt, sl, po, li, j0, vv);
#pragma unroll
      for (int u = 0; u < 8; ++u) xx[u] = x[cc[u]];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const T w = (j0 + u < sl.width) ? vv[u] : T(0);
        acc += w * xx[u];
      }
    }
    acc += (V.dcode ? dt[dcode] : dval) * xp;
    if (lane < sl.nrows) {
      if (MODE == 0) {
        s[p] = rp - acc;
      } else {
        s[p] = acc;
        if (MODE == 1) dsum = (double)xp * (double)acc;
      }
    }
  }
  if (MODE == 1) block_partials<1>(dsum, 0.0, red.part);
}

// ------------------------------------------------------ grouped levels

// Grouped levels: one wavefront per group, LPR = 64 / KMAX lanes per row
// (KMAX a power of two, at least the level's largest group).  Every group has
// a 96-byte record (read by the lanes, word t in lane t, and taken apart with
// readlane):
//   rec[0] first row p0, rec[1] rows k, rec[2] offset of its k x k diagonal
//   block (dense row-major), rec[3 + q] entry offset of row q (q = 0..8,
//   repeated past row k), rec[12 + q] (q < 8) the end of row q's entries in
//   earlier smoother stages (a row's entries are in increasing column order),
//   rec[20] and rec[21]: entry e of row q has its column index at
//   col[e + rec[20] - q rec[21]] (rec[21] is the row length when the rows
//   share one stored column list, else 0), rec[22..23] unused.
// In the forward sweep from x = 0 (first = 1) the rows are summed only up to
// that end: the entries of later stages multiply values that are still zero.
// Lane sub of row l strides over row l's off-group entries (batches of 4:
// index loads, gathers, sums); the row is summed inside its aligned group of
// lanes with DPP moves and each row sum is read into a scalar with readlane.
constexpr int kRec = 24;

// The group's record, diagonal block, and current x and r of its rows, as
// the block-per-group kernels hold them (indices clamped into the group).
template <typename T, int KMAX>
struct GroupData {
  int p0, k, cs, cm;  // cs, cm: rec[20], rec[21]
  int gb[kKmax + 1];
  T B[KMAX][KMAX], xv[KMAX], rv[KMAX];
};

// One Gauss-Seidel stage on the groups [g0, g1): every group relaxes its rows
// one after the other (forward: l = 0..k-1, backward: l = k-1..0) with the
// latest values of the other rows.  The record is read by the lanes (lane t
// holds word t) and its uniform fields taken with readlane: one vector load
// and one wait, after which the diagonal block, x and r of the rows and the
// row entries are all requested together; they reach every lane by readlane
// once the row sums are done.  The dependent chain is record -> entries and
// group data -> neighbour values -> store.
template <typename T, int KMAX, int BACK>
__global__ __launch_bounds__(kBlock) void k_gs_grp(int g0, int g1, const int* __restrict__ rec,
                                                   const int* __restrict__ col, const T* __restrict__ val,
                                                   const T* __restrict__ dblk, const T* __restrict__ r, T* x,
                                                   int first) {
  constexpr int LPR = 64 / KMAX;
  const int graw = g0 + xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (int)(threadIdx.x >> 6);
  const int g = __builtin_amdgcn_readfirstlane(min(graw, g1 - 1));
  const int lane = threadIdx.x & 63;
  const int l = lane / LPR, sub = lane % LPR;
  const int rw = rec[(size_t)g * kRec + min(lane, kRec - 1)];
  const int p0 = __builtin_amdgcn_readlane(rw, 0), k = __builtin_amdgcn_readlane(rw, 1);
  const int boff = __builtin_amdgcn_readlane(rw, 2);
  const int csh = __builtin_amdgcn_readlane(rw, 20) - l * __builtin_amdgcn_readlane(rw, 21);
  int e0 = __builtin_amdgcn_readlane(rw, 3), e1 = __builtin_amdgcn_readlane(rw, 4);
  int sp = __builtin_amdgcn_readlane(rw, 12);
#pragma unroll
  for (int q = 1; q < KMAX; ++q)
    if (l == q) {
      e0 = __builtin_amdgcn_readlane(rw, 3 + q);
      e1 = __builtin_amdgcn_readlane(rw, 4 + q);
      sp = __builtin_amdgcn_readlane(rw, 12 + q);
    }
  if (first) e1 = sp;  // forward sweep from zero: entries of earlier stages only
  // group data: lane t < KMAX^2 the block entry (t / KMAX, t % KMAX), lane t
  // < KMAX row t's x and r (indices clamped into the group)
  const int tb = min(lane, KMAX * KMAX - 1);
  const T bq = dblk[boff + min(tb / KMAX, k - 1) * k + min(tb % KMAX, k - 1)];
  const T xo = x[p0 + min(lane, k - 1)];
  const T ro = r[p0 + min(lane, k - 1)];
  T acc = T(0);
  for (int e = e0 + sub; e < e1; e += 4 * LPR) {
    int cc[4];
    T vv[4], xx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ee = min(e + u * LPR, e1 - 1);
      cc[u] = col[ee + csh];
      vv[u] = val[ee];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) xx[u] = x[cc[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (e + u * LPR < e1) acc += vv[u] * xx[u];
  }
  acc = lanes_sum<LPR>(acc);
  T a[KMAX], B[KMAX][KMAX], xv[KMAX], dinv[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    T t = lane_value(acc, q * LPR);
#pragma unroll
    for (int j = 1; j < LPR / 16; ++j) t += lane_value(acc, q * LPR + 16 * j);
    a[q] = t;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) B[q][j] = lane_value(bq, q * KMAX + j);
    xv[q] = (q < k) ? lane_value(xo, q) : T(0);
    a[q] = (q < k) ? lane_value(ro, q) - a[q] : T(0);  // r minus the off-group sum
    dinv[q] = T(1) / B[q][q];
  }
#pragma unroll
  for (int t = 0; t < KMAX; ++t) {
    const int ll = BACK ? KMAX - 1 - t : t;
    if (ll < k) {
      T s = a[ll];
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q < k && q != ll) s -= B[ll][q] * xv[q];
      xv[ll] = s * dinv[ll];
    }
  }
  if (graw < g1 && sub == 0 && l < k) {
    T v = xv[0];
#pragma unroll
    for (int q = 1; q < KMAX; ++q)
      if (l == q) v = xv[q];
    x[p0 + l] = v;
  }
}

// Forward sweep from x = 0 on a grouped level: the groups of stage 0 solve
// their lower-triangular block (the rest of the row multiplies zeros); all
// other rows are zeroed.  One thread per group.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_zero_stage0_grp(int ng, int ng0, const int* __restrict__ gstart,
                                                            const int* __restrict__ dboff, const T* __restrict__ dblk,
                                                            const T* __restrict__ r, T* __restrict__ x) {
  for (int g = blockIdx.x * kBlock + threadIdx.x; g < ng; g += gridDim.x * kBlock) {
    const int p0 = gstart[g], k = gstart[g + 1] - p0;
    if (g >= ng0) {
      for (int q = 0; q < k; ++q) x[p0 + q] = T(0);
      continue;
    }
    const T* B = dblk + dboff[g];
    T xv[kKmax];
#pragma unroll
    for (int l = 0; l < kKmax; ++l) {
      xv[l] = T(0);
      if (l < k) {
        T s = r[p0 + l];
#pragma unroll
        for (int q = 0; q < kKmax; ++q)
          if (q < l) s -= B[l * k + q] * xv[q];
        xv[l] = s / B[l * k + l];
      }
    }
#pragma unroll
    for (int q = 0; q < kKmax; ++q)
      if (q < k) x[p0 + q] = xv[q];
  }
}

// s = r - A x (MODE 0), y = A x with sum x.y (MODE 1, binary64) or y = A x
// (MODE 2) on all groups; wave per group.  Loads as in k_gs_grp: the record
// by the lanes, then the block, x of the rows, r of the lane's row and the
// entries together, then the neighbour values.
template <typename T, int KMAX, int MODE>
__global__ __launch_bounds__(kBlock) void k_resid_grp(int ng, const int* __restrict__ rec,
                                                      const int* __restrict__ col, const T* __restrict__ val,
                                                      const T* __restrict__ dblk, const T* __restrict__ r,
                                                      const T* __restrict__ x, T* __restrict__ s, Red red) {
  constexpr int LPR = 64 / KMAX;
  const int graw = xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (int)(threadIdx.x >> 6);
  const int g = __builtin_amdgcn_readfirstlane(min(graw, ng - 1));
  const int lane = threadIdx.x & 63;
  const int l = lane / LPR, sub = lane % LPR;
  const int rw = rec[(size_t)g * kRec + min(lane, kRec - 1)];
  const int p0 = __builtin_amdgcn_readlane(rw, 0), k = __builtin_amdgcn_readlane(rw, 1);
  const int boff = __builtin_amdgcn_readlane(rw, 2);
  const int csh = __builtin_amdgcn_readlane(rw, 20) - l * __builtin_amdgcn_readlane(rw, 21);
  int e0 = __builtin_amdgcn_readlane(rw, 3), e1 = __builtin_amdgcn_readlane(rw, 4);
#pragma unroll
  for (int q = 1; q < KMAX; ++q)
    if (l == q) {
      e0 = __builtin_amdgcn_readlane(rw, 3 + q);
      e1 = __builtin_amdgcn_readlane(rw, 4 + q);
    }
  const int tb = min(lane, KMAX * KMAX - 1);
  const T bq = dblk[boff + min(tb / KMAX, k - 1) * k + min(tb % KMAX, k - 1)];
  const T xo = x[p0 + min(lane, k - 1)];
  const int pl = p0 + min(l, k - 1);
  const T rl = MODE == 0 ? r[pl] : T(0);
  T acc = T(0);
  for (int e = e0 + sub; e < e1; e += 4 * LPR) {
    int cc[4];
    T vv[4], xx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ee = min(e + u * LPR, e1 - 1);
      cc[u] = col[ee + csh];
      vv[u] = val[ee];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) xx[u] = x[cc[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (e + u * LPR < e1) acc += vv[u] * xx[u];
  }
  acc = lanes_sum<LPR>(acc);
  // this lane's row l: its off-group sum, then the diagonal block's terms
  T t = T(0), xl = T(0);
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    T aq = lane_value(acc, q * LPR);
#pragma unroll
    for (int j = 1; j < LPR / 16; ++j) aq += lane_value(acc, q * LPR + 16 * j);
    const T xq = lane_value(xo, q);
    if (q == l) {
      t = aq;
      xl = xq;
    }
  }
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    T bl = lane_value(bq, q);  // row 0
#pragma unroll
    for (int i = 1; i < KMAX; ++i)
      if (i == l) bl = lane_value(bq, i * KMAX + q);
    if (q < k) t += bl * lane_value(xo, q);
  }
  double dsum = 0.0;
  if (graw < ng && sub == 0 && l < k) {
    const int p = p0 + l;
    if (MODE == 0) {
      s[p] = rl - t;
    } else {
      s[p] = t;
      if (MODE == 1) dsum = (double)xl * (double)t;
    }
  }
  if (MODE == 1) block_partials<1>(dsum, 0.0, red.part);
}

// --------------------------------------------------- wide grouped kernels

// Levels whose groups carry many entries (long rows, few groups per stage):
// one block of NT threads per group (kWide for a smoother stage, which covers
// few groups; kWideResid for a residual, which covers all of them).  Row l of
// the group takes the NT / KMAX lanes l * NT / KMAX ..; every lane adds its
// entries four at a time (their loads in flight together).  The lanes of a
// row are summed in segments of up to 64 (DPP, then readlane), the segment
// sums go to LDS and a row's segments are added in order.  The rest is as in
// k_gs_grp and k_resid_grp.
constexpr int kWide = 1024, kWideResid = 256;

template <typename T, int KMAX, int NT>
__device__ __forceinline__ void wide_rowsums(const GroupData<T, KMAX>& d, const int* __restrict__ col,
                                             const T* __restrict__ val, const T* x, T (&a)[KMAX],
                                             const int* __restrict__ split = nullptr) {
  constexpr int LPR = NT / KMAX;                // lanes per row
  constexpr int SEG = LPR < 64 ? LPR : 64;      // lanes per segment sum
  constexpr int SPR = LPR / SEG;                // segments per row
  static_assert(SEG >= 16, "at least 16 lanes per row");
  __shared__ T red[NT / SEG];
  const int l = (int)threadIdx.x / LPR, sub = (int)threadIdx.x % LPR;
  T acc = T(0);
  if (l < d.k) {
    int e0 = d.gb[0], e1 = d.gb[1];
#pragma unroll
    for (int q = 1; q < KMAX; ++q)
      if (q == l) {
        e0 = d.gb[q];
        e1 = d.gb[q + 1];
      }
    if (split) e1 = split[min(l, kKmax - 1)];
    const int csh = d.cs - l * d.cm;
    for (int e = e0 + sub; e < e1; e += 4 * LPR) {
      int cc[4];
      T vv[4], xx[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int ee = e + u * LPR;
        const bool ok = ee < e1;
        const int es = ok ? ee : e;
        cc[u] = col[es + csh];
        vv[u] = ok ? val[es] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) xx[u] = x[cc[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += vv[u] * xx[u];
    }
  }
  acc = lanes_sum<16>(acc);
  const int lane = threadIdx.x & 63;
  if (SEG == 64) {
    acc = ((lane_value(acc, 0) + lane_value(acc, 16)) + lane_value(acc, 32)) + lane_value(acc, 48);
  } else if (SEG == 32) {
    const T h0 = lane_value(acc, 0) + lane_value(acc, 16), h1 = lane_value(acc, 32) + lane_value(acc, 48);
    acc = (lane < 32) ? h0 : h1;
  }
  if (((int)threadIdx.x % SEG) == 0) red[threadIdx.x / SEG] = acc;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    T t = red[q * SPR];
#pragma unroll
    for (int i = 1; i < SPR; ++i) t += red[q * SPR + i];
    a[q] = t;
  }
}

// Group data for a block-per-group kernel: the record with scalar loads, the
// diagonal block, x and r of the group once per block into LDS (threads
// t < KMAX * KMAX and t < KMAX); visible after the block's next barrier, and
// read back by the first wave only, which finishes the group.
template <typename T, int KMAX, bool WITH_R>
struct WideStage {
  T B[KMAX * KMAX], xv[KMAX], rv[KMAX];
};

template <typename T, int KMAX, bool WITH_R>
__device__ __forceinline__ void wide_load_group(int g, const int* __restrict__ rec, const T* __restrict__ dblk,
                                                const T* __restrict__ r, const T* x, GroupData<T, KMAX>& d,
                                                WideStage<T, KMAX, WITH_R>& st) {
  const int* R = rec + (size_t)g * kRec;
  d.p0 = R[0];
  d.k = R[1];
  d.cs = R[20];
  d.cm = R[21];
  const int db = R[2];
#pragma unroll
  for (int q = 0; q <= kKmax; ++q) d.gb[q] = R[3 + q];
  const int k = d.k, t = threadIdx.x;
  if (t < KMAX * KMAX) st.B[t] = dblk[db + min(t / KMAX, k - 1) * k + min(t % KMAX, k - 1)];
  if (t < KMAX) {
    const T xi = x[d.p0 + min(t, k - 1)];
    st.xv[t] = (t < k) ? xi : T(0);
    if (WITH_R) {
      const T ri = r[d.p0 + min(t, k - 1)];
      st.rv[t] = (t < k) ? ri : T(0);
    }
  }
}

template <typename T, int KMAX, int BACK>
__global__ __launch_bounds__(kWide) void k_gs_grp_wide(int g0, int g1, const int* __restrict__ rec,
                                                       const int* __restrict__ col, const T* __restrict__ val,
                                                       const T* __restrict__ dblk, const T* __restrict__ r, T* x,
                                                       int first) {
  const int g = g0 + xcd_block(blockIdx.x, gridDim.x);
  GroupData<T, KMAX> d;
  __shared__ WideStage<T, KMAX, true> st;
  wide_load_group<T, KMAX, true>(g, rec, dblk, r, x, d, st);
  T a[KMAX];
  wide_rowsums<T, KMAX, kWide>(d, col, val, x, a, first ? rec + (size_t)g * kRec + 12 : nullptr);  // ends with a barrier
  if (threadIdx.x >= 64) return;  // the first wave solves the group's rows
  // the block stays in LDS; x and r of the group in registers
  T xv[KMAX], rv[KMAX], dinv[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    xv[q] = st.xv[q];
    rv[q] = st.rv[q];
    dinv[q] = T(1) / st.B[q * KMAX + q];
  }
#pragma unroll
  for (int t = 0; t < KMAX; ++t) {
    const int ll = BACK ? KMAX - 1 - t : t;
    if (ll < d.k) {
      T s = rv[ll] - a[ll];
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q < d.k && q != ll) s -= st.B[ll * KMAX + q] * xv[q];
      xv[ll] = s * dinv[ll];
    }
  }
  const int l = threadIdx.x;
  if (l < d.k) {
    T v = xv[0];
#pragma unroll
    for (int q = 1; q < KMAX; ++q)
      if (l == q) v = xv[q];
    x[d.p0 + l] = v;
  }
}

// s = r - A x on the groups [0, ng), one block per group.
template <typename T, int KMAX>
__global__ __launch_bounds__(kWideResid) void k_resid_grp_wide(int ng, const int* __restrict__ rec,
                                                          const int* __restrict__ col, const T* __restrict__ val,
                                                          const T* __restrict__ dblk, const T* __restrict__ r,
                                                          const T* __restrict__ x, T* __restrict__ s) {
  const int g = xcd_block(blockIdx.x, gridDim.x);
  GroupData<T, KMAX> d;
  __shared__ WideStage<T, KMAX, false> st;
  wide_load_group<T, KMAX, false>(g, rec, dblk, r, x, d, st);
  T a[KMAX];
  wide_rowsums<T, KMAX, kWideResid>(d, col, val, x, a);  // ends with a barrier
  if (threadIdx.x >= 64) return;  // the first wave finishes the group's rows
  const int l = threadIdx.x;
  if (l < d.k) {
    T t = a[0];
#pragma unroll
    for (int q = 1; q < KMAX; ++q)
      if (q == l) t = a[q];
    // row l of the block from LDS, x of the group in order
#pragma unroll
    for (int q = 0; q < KMAX; ++q)
      if (q < d.k) t += st.B[l * KMAX + q] * st.xv[q];
    const int p = d.p0 + l;
    s[p] = r[p] - t;
  }
}

// ------------------------------------------------------------ l1-Jacobi

template <typename T>
__global__ __launch_bounds__(kBlock) void k_l1_init(int n, const T* __restrict__ dl1, const T* __restrict__ r,
                                                    T* __restrict__ x) {
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) x[p] = r[p] / dl1[p];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_l1_update(int n, const T* __restrict__ dl1, const T* __restrict__ s,
                                                      T* __restrict__ x) {
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) x[p] += s[p] / dl1[p];
}

// l1 row norms d_p = sum_j |a_pj| (entries outside and inside the diagonal block)
__global__ __launch_bounds__(kBlock) void k_l1norm_sell(const Slab* __restrict__ slabs, int nslabs,
                                                        const double* __restrict__ val, const double* __restrict__ diag,
                                                        double* __restrict__ dl1) {
  const int sidx = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (sidx >= nslabs) return;
  const Slab sl = slabs[sidx];
  if (lane >= sl.nrows) return;
  double a = fabs(diag[sl.row0 + lane]);
  for (int j = 0; j < sl.width; ++j) a += fabs(val[sl.off + 64 * j + lane]);
  dl1[sl.row0 + lane] = a;
}

__global__ __launch_bounds__(kBlock) void k_l1norm_grp(int ng, const int* __restrict__ gstart,
                                                       const int* __restrict__ rowptr, const double* __restrict__ val,
                                                       const int* __restrict__ dboff, const double* __restrict__ dblk,
                                                       double* __restrict__ dl1) {
  for (int g = blockIdx.x * kBlock + threadIdx.x; g < ng; g += gridDim.x * kBlock) {
    const int p0 = gstart[g], k = gstart[g + 1] - p0;
    for (int l = 0; l < k; ++l) {
      double a = 0.0;
      for (int e = rowptr[p0 + l]; e < rowptr[p0 + l + 1]; ++e) a += fabs(val[e]);
      for (int q = 0; q < k; ++q) a += fabs(dblk[dboff[g] + l * k + q]);
      dl1[p0 + l] = a;
    }
  }
}

// ------------------------------------------------------------- transfers

// Per-aggregate record of a transfer, kARec ints: first entry of the
// aggregate's members in arows, member count n_a, block width k, offset of
// U_a, first coarse row, and the offset of the aggregate's k x k diagonal
// block on the next level when that level is smoothed by Gauss-Seidel and
// the aggregate's group there belongs to stage 0 (-1 otherwise).  One record
// replaces the chain aggregate -> group -> block offset -> block.
constexpr int kARec = 8;
enum ARecField { AR_M0 = 0, AR_NA = 1, AR_K = 2, AR_UOFF = 3, AR_C0 = 4, AR_DB = 5 };

// r_c = P^T s with P = blockdiag(U_a): LPA lanes per aggregate (16: one DPP
// row, four aggregates per wave; 64: one wave), lane g takes members g,
// g + LPA, ... four at a time, all their loads in flight together;
// r_c[c0 + l] = sum_li U_a[li, l] s[member li].  U_a is stored column-major
// (U[l * n_a + li]), members in increasing row order; KMAX bounds the block
// widths k.  Rows >= scut have s = 0: neither s nor U is read for them.
//
// The k coarse rows of an aggregate are one smoother group of the next level,
// so the kernel can also start that level's pre-smoothing from x_c = 0
// (INIT = 1: the groups of stage 0 solve their lower-triangular diagonal block,
// the others are zero -- the first Gauss-Seidel stage; INIT = 2: x_c = r_c / d_l1,
// the first l1-Jacobi sweep).  The record, then U_a, the member rows and the
// diagonal block's lower triangle are all requested before the gathers of s.
template <typename T, int KMAX, int INIT, int LPA>
__global__ __launch_bounds__(kBlock) void k_restrict(int nagg, const int* __restrict__ arec,
                                                     const int* __restrict__ arows, const T* __restrict__ U,
                                                     const T* __restrict__ s, int scut, T* __restrict__ rc,
                                                     const T* __restrict__ cdblk, const T* __restrict__ cdl1,
                                                     T* __restrict__ xc, Skip sk) {
  const int g = threadIdx.x & (LPA - 1);
  const int a = (xcd_block(blockIdx.x, gridDim.x) * kBlock + (int)threadIdx.x) / LPA;
  const bool on = a < nagg && !skipped(sk, a);
  const int* R = arec + (size_t)min(a, nagg - 1) * kARec;
  const int m0 = R[AR_M0], na = on ? R[AR_NA] : 0, k = R[AR_K], c0 = R[AR_C0];
  const T* Ua = U + R[AR_UOFF];
  // lower triangle of the diagonal block (indices clamped into the k x k
  // block; a record without a block reads the level's first block, which is
  // at least k x k, and discards it)
  constexpr int NB = (INIT == 1) ? KMAX * (KMAX + 1) / 2 : 1;
  T bl[NB];
  int db = -1;
  if (INIT == 1) {
    db = R[AR_DB];
    const T* B = cdblk + max(db, 0);
#pragma unroll
    for (int l = 0; l < KMAX; ++l)
#pragma unroll
      for (int q = 0; q <= l; ++q) bl[l * (l + 1) / 2 + q] = B[min(l, k - 1) * k + min(q, k - 1)];
  }
  T acc[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) acc[q] = T(0);
  for (int b0 = 0; b0 < na; b0 += 4 * LPA) {
    int row[4];
    T u[4][KMAX], sv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int li = b0 + g + v * LPA;
      row[v] = (li < na) ? arows[m0 + li] : INT_MAX;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int li = b0 + g + v * LPA;
      const bool live = row[v] < scut;
#pragma unroll
      for (int q = 0; q < KMAX; ++q) u[v][q] = live ? Ua[min(q, k - 1) * na + li] : T(0);
      sv[v] = live ? s[row[v]] : T(0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q < k) acc[q] += u[v][q] * sv[v];
  }
  // sums over the aggregate's lanes: DPP inside each 16-lane row, then (one
  // aggregate per wave) the four row sums in order
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    const T v = lanes_sum<16>(acc[q]);
    acc[q] = (LPA == 16) ? v : ((lane_value(v, 0) + lane_value(v, 16)) + lane_value(v, 32)) + lane_value(v, 48);
  }
  T out = acc[0];
#pragma unroll
  for (int q = 1; q < KMAX; ++q)
    if (g == q) out = acc[q];
  if (on && g < k) rc[c0 + g] = out;
  if (INIT == 1) {
    T xv[KMAX];
#pragma unroll
    for (int l = 0; l < KMAX; ++l) {
      T tt = acc[l];
#pragma unroll
      for (int q = 0; q < l; ++q) tt -= bl[l * (l + 1) / 2 + q] * xv[q];
      xv[l] = (db >= 0 && l < k) ? tt / bl[l * (l + 1) / 2 + l] : T(0);
    }
    T xo = xv[0];
#pragma unroll
    for (int q = 1; q < KMAX; ++q)
      if (g == q) xo = xv[q];
    if (on && g < k) xc[c0 + g] = xo;
  } else if (INIT == 2) {
    if (on && g < k) xc[c0 + g] = out / cdl1[c0 + g];
  }
}

// x += P x_c in fine-row order (coalesced) on the rows i < n: thread per
// fine row i with cinfo[i] = 8 * (first coarse row of its aggregate) + (k - 1)
// and the row's k entries of U at Urow[q * ld + i] (zero past k).
template <typename T, int KMAX>
__global__ __launch_bounds__(kBlock) void k_prolong_rows(int n, int ld, const int* __restrict__ cinfo,
                                                         const T* __restrict__ Urow, const T* __restrict__ xc,
                                                         T* __restrict__ x, Skip sk) {
  for (int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    if (skipped(sk, i)) continue;
    // x, the record and all KMAX entries of U (zero past k) are requested
    // together; the coarse values past k are read at a clamped index and
    // weighted by those zeros
    const T xi = x[i];
    const int ci = cinfo[i];
    T u[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) u[q] = Urow[(size_t)q * ld + i];
    const int c0 = ci >> 3, k = (ci & 7) + 1;
    T t = T(0);
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      const T v = xc[c0 + min(q, k - 1)];
      t += (q < k ? u[q] : T(0)) * v;
    }
    x[i] = xi + t;
  }
}

// ------------------------------------------------------------- coarsest

// Symmetric A (n x n) as its lower-triangle 64 x 64 tiles: tile t = (I, J),
// J <= I, listed in tij, stored row-major at tiles + 4096 t with every entry
// of a row or column >= n zero; diagonal tiles whole.  Built once from the
// padded row-major matrix A (leading dimension ld).
__global__ __launch_bounds__(kBlock) void k_pack_tiles(int n, int ld, const int2* __restrict__ tij,
                                                       const double* __restrict__ A, double* __restrict__ tiles) {
  const int t = blockIdx.x;
  const int2 ij = tij[t];
  for (int e = threadIdx.x; e < 4096; e += kBlock) {
    const int r = ij.x * 64 + (e >> 6), c = ij.y * 64 + (e & 63);
    tiles[(size_t)t * 4096 + e] = (r < n && c < n) ? A[(size_t)r * ld + c] : 0.0;
  }
}

// y = A x, first pass: tile t = (I, J) adds A_IJ x_J to row block I and, for
// J < I, A_IJ^T x_I to row block J, each into its own slot of part (row
// block R, column block C at part + 64 (R nt + C)); k_symv_sum adds the slots.
// Every tile is read once -- half the bytes of the full product.  Wave w
// takes rows 16 w .. 16 w + 15 of the tile, lane l the columns 2 (l % 32),
// 2 (l % 32) + 1 of rows 16 w + 2 i + l / 32 (i < 8, one 16-byte load each).
__global__ __launch_bounds__(kBlock) void k_symv_tiles(int n, int nt, const int2* __restrict__ tij,
                                                       const double* __restrict__ tiles,
                                                       const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double colp[kBlock / 64][64];
  const int t = blockIdx.x;
  const int2 ij = tij[t];
  const int I = ij.x, J = ij.y;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, h = lane >> 5, cp = 2 * (lane & 31);
  const double* Tt = tiles + (size_t)t * 4096;
  double2 a[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = *reinterpret_cast<const double2*>(Tt + (16 * w + 2 * i + h) * 64 + cp);
  const int cj = J * 64 + cp;
  const double xj0 = (cj < n) ? x[cj] : 0.0, xj1 = (cj + 1 < n) ? x[cj + 1] : 0.0;
  double xi[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int ri = I * 64 + 16 * w + 2 * i + h;
    xi[i] = (ri < n) ? x[ri] : 0.0;
  }
  // row sums: DPP inside the 16-lane rows, then the two rows of each half wave
  double out = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double v = lanes_sum<16>(a[i].x * xj0 + a[i].y * xj1);
    const double s0 = lane_value(v, 0) + lane_value(v, 16), s1 = lane_value(v, 32) + lane_value(v, 48);
    if (lane == 2 * i) out = s0;
    if (lane == 2 * i + 1) out = s1;
  }
  if (lane < 16) part[((size_t)I * nt + J) * 64 + 16 * w + lane] = out;
  if (J < I) {
    // column sums over the wave's rows, then over the four waves in order
    double c0 = 0.0, c1 = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      c0 += a[i].x * xi[i];
      c1 += a[i].y * xi[i];
    }
    c0 += __shfl_xor(c0, 32, 64);
    c1 += __shfl_xor(c1, 32, 64);
    if (h == 0) {
      colp[w][cp] = c0;
      colp[w][cp + 1] = c1;
    }
    __syncthreads();
    if (w == 0) part[((size_t)J * nt + I) * 64 + lane] = ((colp[0][lane] + colp[1][lane]) + colp[2][lane]) + colp[3][lane];
  }
}

// y = A x, second pass, one block per row block R: wave w adds the slots of
// the column blocks in its quarter [w q, (w + 1) q), eight loads in flight,
// and the four quarter sums are added in order.
__global__ __launch_bounds__(kBlock) void k_symv_sum(int n, int nt, const double* __restrict__ part,
                                                     double* __restrict__ y) {
  __shared__ double red[kBlock / 64][64];
  const int R = blockIdx.x, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = (nt + 3) / 4, c0 = w * q, c1 = min(nt, c0 + q);
  const double* p = part + (size_t)R * nt * 64 + lane;
  double s = 0.0;
  for (int c = c0; c < c1; c += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(size_t)min(c + u, c1 - 1) * 64];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (c + u < c1) s += v[u];
  }
  red[w][lane] = s;
  __syncthreads();
  const int i = R * 64 + lane;
  if (w == 0 && i < n) y[i] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// ------------------------------------------------- values, casts, gradient

// flag[0] = 1 if a and b differ in any of their n entries (several threads
// may store the same 1).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_differs(int64_t n, const T* __restrict__ a, const T* __restrict__ b,
                                                    int* __restrict__ flag) {
  bool d = false;
  for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock)
    d |= (a[e] != b[e]);
  if (d) flag[0] = 1;
}

// dst[e] = src_idx[e] >= 0 ? val[src_idx[e]] : 0 (layout fill from file-order values)
__global__ __launch_bounds__(kBlock) void k_fill_values(int64_t m, const int* __restrict__ src,
                                                        const double* __restrict__ val, double* __restrict__ dst) {
  for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kBlock) {
    const int s = src[e];
    dst[e] = (s >= 0) ? val[s] : 0.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_to_f32(int64_t m, const double* __restrict__ in, float* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kBlock)
    out[e] = (float)in[e];
}

// dval[e] = -lambda_i x_j for the stored entries (i, j) of a CSR pattern
__global__ __launch_bounds__(kBlock) void k_grad_coeffs(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                        const double* __restrict__ lam, const double* __restrict__ x,
                                                        double* __restrict__ dval) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double li = lam[i];
    for (int e = rp[i]; e < rp[i + 1]; ++e) dval[e] = -li * x[ci[e]];
  }
}

}  // namespace mvamg
