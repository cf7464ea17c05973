// Numeric setup of one multiple-vector level on the device (Section 4): the
// per-aggregate local bases of eq. 4.3, the Galerkin product
// A_c = P^T A P with P = blockdiag(U_a), and the smooth vectors restricted
// to the coarse level (Section 4.1).
#pragma once

#include "kernels.hpp"

namespace mvamg {

// Bases: one wave per aggregate.  The n_a x m block of the smooth vectors
// sits in LDS (row-major); lane t owns rows t, t + 64, ...  One-sided Jacobi
// (Hestenes) rotates column pairs until every pair is orthogonal to working
// precision; the column norms are the singular values and the normalised
// columns the left singular vectors.
constexpr int kSvdMaxM = 16;
constexpr int kSvdSweeps = 60;

// sum over the wave of (v, index) pairs: the largest |v|, the lowest index on ties
__device__ __forceinline__ int wave_argmax_abs(double v, int idx) {
  double best = fabs(v);
  int bi = idx;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ov > best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
    }
  }
  return bi;
}

__global__ __launch_bounds__(64) void k_setup_bases(int m, int nagg, const int* __restrict__ aptr,
                                                    const int* __restrict__ arows, const double* __restrict__ W,
                                                    double tol_per_row, int* __restrict__ kout,
                                                    double* __restrict__ U, double* __restrict__ dropped,
                                                    int* __restrict__ flag) {
  extern __shared__ double G[];  // n_a x m of this aggregate
  const int a = blockIdx.x;
  if (a >= nagg) return;
  const int lane = threadIdx.x;
  const int r0 = aptr[a], na = aptr[a + 1] - r0;
  for (int i = lane; i < na; i += 64) {
    const int row = arows[r0 + i];
    for (int c = 0; c < m; ++c) G[i * m + c] = W[(size_t)row * m + c];
  }
  // every lane reads only its own rows from here on: no barrier needed
  for (int sweep = 0; sweep < kSvdSweeps; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < na; i += 64) {
          const double gp = G[i * m + p], gq = G[i * m + q];
          al += gp * gp;
          be += gq * gq;
          ga += gp * gq;
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
        rotated = true;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
        for (int i = lane; i < na; i += 64) {
          const double gp = G[i * m + p], gq = G[i * m + q];
          G[i * m + p] = cs * gp - sn * gq;
          G[i * m + q] = sn * gp + cs * gq;
        }
      }
    if (!rotated) break;
  }
  double sig[kSvdMaxM];
  int ord[kSvdMaxM];
  for (int c = 0; c < m; ++c) {
    double s = 0.0;
    for (int i = lane; i < na; i += 64) s += G[i * m + c] * G[i * m + c];
    sig[c] = sqrt(wave_sum(s));
    ord[c] = c;
  }
  // descending singular values, stable in the column index (every lane the same)
  for (int i = 1; i < m; ++i) {
    const int v = ord[i];
    int j = i - 1;
    while (j >= 0 && sig[ord[j]] < sig[v]) {
      ord[j + 1] = ord[j];
      --j;
    }
    ord[j + 1] = v;
  }
  const double tol_a = tol_per_row * na;
  int k = 0;
  while (k < m && k < na && sig[ord[k]] > tol_a) ++k;
  if (k == 0) k = 1;
  if (!(sig[ord[0]] > 0.0) && lane == 0) flag[0] = 1;
  double drop = 0.0;
  for (int l = k; l < m; ++l) drop += sig[ord[l]] * sig[ord[l]];
  for (int l = 0; l < k; ++l) {
    const int c = ord[l];
    const double inv = sig[c] > 0.0 ? 1.0 / sig[c] : 0.0;
    // the sign rule: the entry of largest magnitude (lowest row on ties) positive
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = lane; i < na; i += 64) {
      const double v = fabs(G[i * m + c]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    const int im = wave_argmax_abs(best < 0.0 ? 0.0 : best, bi);
    const double sgn = (G[im * m + c] < 0.0) ? -inv : inv;
    for (int i = lane; i < na; i += 64) U[(size_t)(r0 + i) * m + l] = G[i * m + c] * sgn;
  }
  for (int l = k; l < m; ++l)
    for (int i = lane; i < na; i += 64) U[(size_t)(r0 + i) * m + l] = 0.0;
  if (lane == 0) {
    kout[a] = k;
    dropped[a] = drop;
  }
}

// W_c[coff[a] + l][r] = sum over the members i of a of U_a[i][l] W[arows[i]][r]
// (one wave per aggregate, lane = (l, r) pair)
__global__ __launch_bounds__(64) void k_setup_restrict(int m, int nagg, const int* __restrict__ aptr,
                                                       const int* __restrict__ arows, const int* __restrict__ coff,
                                                       const double* __restrict__ U, const double* __restrict__ W,
                                                       double* __restrict__ Wc) {
  const int a = blockIdx.x;
  if (a >= nagg) return;
  const int r0 = aptr[a], na = aptr[a + 1] - r0, k = coff[a + 1] - coff[a];
  for (int t = threadIdx.x; t < k * m; t += 64) {
    const int l = t / m, r = t % m;
    double s = 0.0;
    for (int i = 0; i < na; ++i) s += U[(size_t)(r0 + i) * m + l] * W[(size_t)arows[r0 + i] * m + r];
    Wc[(size_t)(coff[a] + l) * m + r] = s;
  }
}

// Galerkin values: one wave per aggregate a.  The k_a rows of a share one
// coarse column list (the dofs of the aggregates coupled to a); lane t takes
// the columns t, t + 64, ...  For column C (dof mm of aggregate b) and every
// l < k_a it sums U_a[i][l] a_ij U_b[loc_j][mm] over the fine entries (i, j)
// with i in a and j in b, rows in member order and entries in CSR order.
__global__ __launch_bounds__(64) void k_setup_galerkin(
    int m, int nagg, const int* __restrict__ aptr, const int* __restrict__ arows, const int* __restrict__ coff,
    const int* __restrict__ agg, const int* __restrict__ loc, const int* __restrict__ cagg,
    const int* __restrict__ rowptr, const int* __restrict__ col, const double* __restrict__ val,
    const double* __restrict__ U, const int* __restrict__ crp, const int* __restrict__ ccol,
    double* __restrict__ cval) {
  const int a = blockIdx.x;
  if (a >= nagg) return;
  const int r0 = aptr[a], na = aptr[a + 1] - r0, ka = coff[a + 1] - coff[a];
  const int I0 = coff[a], c0 = crp[I0], len = crp[I0 + 1] - c0;
  for (int t = threadIdx.x; t < len; t += 64) {
    const int C = ccol[c0 + t];
    const int b = cagg[C], mm = C - coff[b];
    double acc[kSvdMaxM];
    for (int l = 0; l < ka; ++l) acc[l] = 0.0;
    for (int li = 0; li < na; ++li) {
      const int i = arows[r0 + li];
      for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const int j = col[e];
        if (agg[j] != b) continue;
        const double w = val[e] * U[(size_t)(aptr[b] + loc[j]) * m + mm];
        for (int l = 0; l < ka; ++l) acc[l] += U[(size_t)(r0 + li) * m + l] * w;
      }
    }
    for (int l = 0; l < ka; ++l) cval[crp[I0 + l] + t] = acc[l];
  }
}

// The same values for levels with few, large aggregates: one block of
// kGalWaves waves per aggregate.  Wave w takes the w-th of kGalWaves
// contiguous runs of a's member rows and sums over them as above; the runs'
// sums go to LDS and are added in run order.  (Each value is then a sum of
// kGalWaves ordered partial sums instead of one running sum: the same terms,
// rounded in another grouping.)
constexpr int kGalWaves = 4;
constexpr int kGalSplitBelow = 8192;  // aggregates

__global__ __launch_bounds__(64 * kGalWaves) void k_setup_galerkin_split(
    int m, int nagg, const int* __restrict__ aptr, const int* __restrict__ arows, const int* __restrict__ coff,
    const int* __restrict__ agg, const int* __restrict__ loc, const int* __restrict__ cagg,
    const int* __restrict__ rowptr, const int* __restrict__ col, const double* __restrict__ val,
    const double* __restrict__ U, const int* __restrict__ crp, const int* __restrict__ ccol,
    double* __restrict__ cval) {
  __shared__ double part[kGalWaves][kSvdMaxM][64];
  const int a = blockIdx.x;
  if (a >= nagg) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r0 = aptr[a], na = aptr[a + 1] - r0, ka = coff[a + 1] - coff[a];
  const int I0 = coff[a], c0 = crp[I0], len = crp[I0 + 1] - c0;
  const int li0 = (int)((int64_t)na * w / kGalWaves), li1 = (int)((int64_t)na * (w + 1) / kGalWaves);
  for (int t0 = 0; t0 < len; t0 += 64) {
    const int t = t0 + lane;
    double acc[kSvdMaxM];
#pragma unroll
    for (int l = 0; l < kSvdMaxM; ++l) acc[l] = 0.0;
    if (t < len) {
      const int C = ccol[c0 + t];
      const int b = cagg[C], mm = C - coff[b];
      for (int li = li0; li < li1; ++li) {
        const int i = arows[r0 + li];
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
          const int j = col[e];
          if (agg[j] != b) continue;
          const double wv = val[e] * U[(size_t)(aptr[b] + loc[j]) * m + mm];
#pragma unroll
          for (int l = 0; l < kSvdMaxM; ++l)
            if (l < ka) acc[l] += U[(size_t)(r0 + li) * m + l] * wv;
        }
      }
    }
#pragma unroll
    for (int l = 0; l < kSvdMaxM; ++l) part[w][l][lane] = acc[l];
    __syncthreads();
    if (w == 0 && t < len)
#pragma unroll
      for (int l = 0; l < kSvdMaxM; ++l)
        if (l < ka) {
          double v = part[0][l][lane];
#pragma unroll
          for (int q = 1; q < kGalWaves; ++q) v += part[q][l][lane];
          cval[crp[I0 + l] + t] = v;
        }
    __syncthreads();
  }
}

// out_IJ = (in_IJ + in_JI) / 2 over a structurally symmetric CSR with sorted
// rows (the entry J I found by binary search): exactly symmetric.
__global__ __launch_bounds__(kBlock) void k_symmetrize(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const double* __restrict__ in, double* __restrict__ out,
                                                       int* __restrict__ flag) {
  for (int I = blockIdx.x * kBlock + threadIdx.x; I < n; I += gridDim.x * kBlock)
    for (int e = rp[I]; e < rp[I + 1]; ++e) {
      const int J = ci[e];
      int lo = rp[J], hi = rp[J + 1] - 1, f = -1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int c = ci[mid];
        if (c == I) {
          f = mid;
          break;
        }
        if (c < I)
          lo = mid + 1;
        else
          hi = mid - 1;
      }
      if (f < 0) {
        flag[0] = 1;
        out[e] = in[e];
      } else {
        out[e] = (in[e] + in[f]) * 0.5;
      }
    }
}

}  // namespace mvamg
