// Dense kernels for the coarsest level (run once, at upload): blocked
// Cholesky factorisation A = L L^T and the explicit inverse
// A^{-1} = L^{-T} L^{-1}, used by the solve as one matrix-vector product
// (Section 5 solves the coarsest system with a direct method).
//
// The matrix is row-major np x np with np a multiple of 64, padded with the
// identity beyond the true size, so every tile is full.  Tiles of 64 x 64
// binary64 values are staged in LDS (33 KB each with one padding column); a
// 256-thread block computes a 4 x 4 patch per thread.
#pragma once

#include <hip/hip_runtime.h>

namespace mvamg {

constexpr int TD = 64;

__device__ __forceinline__ void load_tile(double (*S)[TD + 1], const double* M, int np, int ti, int tj) {
  const double* A = M + (size_t)ti * TD * np + (size_t)tj * TD;
  for (int e = threadIdx.x; e < TD * TD; e += blockDim.x) {
    const int r = e / TD, c = e % TD;
    S[r][c] = A[(size_t)r * np + c];
  }
}

// Cholesky of the diagonal tile (kb, kb), in place (strict upper part zeroed).
__global__ __launch_bounds__(256) void k_potrf_tile(double* M, int np, int kb, int* flag) {
  __shared__ double T[TD][TD + 1];
  load_tile(T, M, np, kb, kb);
  __syncthreads();
  for (int j = 0; j < TD; ++j) {
    if (threadIdx.x == 0) {
      double d = T[j][j];
      if (!(d > 0.0)) {
        *flag = 1;
        d = 1.0;
      }
      T[j][j] = sqrt(d);
    }
    __syncthreads();
    const double ljj = T[j][j];
    for (int i = j + 1 + (int)threadIdx.x; i < TD; i += blockDim.x) T[i][j] /= ljj;
    __syncthreads();
    for (int e = threadIdx.x; e < TD * TD; e += blockDim.x) {
      const int i = e / TD, l = e % TD;
      if (l > j && l <= i) T[i][l] -= T[i][j] * T[l][j];
    }
    __syncthreads();
  }
  double* A = M + (size_t)kb * TD * np + (size_t)kb * TD;
  for (int e = threadIdx.x; e < TD * TD; e += blockDim.x) {
    const int r = e / TD, c = e % TD;
    A[(size_t)r * np + c] = (c <= r) ? T[r][c] : 0.0;
  }
}

// Panel: L_ik = A_ik L_kk^{-T} for the tiles i = kb+1 .. nb-1 (one block each).
__global__ __launch_bounds__(256) void k_trsm_tile(double* M, int np, int kb) {
  __shared__ double Lk[TD][TD + 1], X[TD][TD + 1];
  const int i = kb + 1 + blockIdx.x;
  load_tile(Lk, M, np, kb, kb);
  load_tile(X, M, np, i, kb);
  __syncthreads();
  for (int j = 0; j < TD; ++j) {
    for (int r = threadIdx.x; r < TD; r += blockDim.x) X[r][j] /= Lk[j][j];
    __syncthreads();
    for (int e = threadIdx.x; e < TD * TD; e += blockDim.x) {
      const int r = e / TD, l = e % TD;
      if (l > j) X[r][l] -= X[r][j] * Lk[l][j];
    }
    __syncthreads();
  }
  double* A = M + (size_t)i * TD * np + (size_t)kb * TD;
  for (int e = threadIdx.x; e < TD * TD; e += blockDim.x) {
    const int r = e / TD, c = e % TD;
    A[(size_t)r * np + c] = X[r][c];
  }
}

// 4 x 4 patch of thread t: rows 4 (t / 16) .., columns 4 (t % 16) ..
// acc += S1 * S2 with S1 indexed [row][m] (or [m][row] when T1) and S2
// indexed [m][col] (or [col][m] when T2).
template <bool T1, bool T2>
__device__ __forceinline__ void tile_mma(const double (*S1)[TD + 1], const double (*S2)[TD + 1],
                                         double (&acc)[4][4]) {
  const int r0 = (threadIdx.x / 16) * 4, c0 = (threadIdx.x % 16) * 4;
  for (int m = 0; m < TD; ++m) {
    double a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = T1 ? S1[m][r0 + q] : S1[r0 + q][m];
      b[q] = T2 ? S2[c0 + q][m] : S2[m][c0 + q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int p = 0; p < 4; ++p) acc[q][p] += a[q] * b[p];
  }
}

// Trailing update A_ij -= L_ik L_jk^T for kb < j <= i < nb (2-D grid; blocks
// above the diagonal return at once).
__global__ __launch_bounds__(256) void k_update_tiles(double* M, int np, int kb) {
  const int i = kb + 1 + blockIdx.y, j = kb + 1 + blockIdx.x;
  if (j > i) return;
  __shared__ double Ai[TD][TD + 1], Aj[TD][TD + 1];
  load_tile(Ai, M, np, i, kb);
  load_tile(Aj, M, np, j, kb);
  __syncthreads();
  double acc[4][4] = {};
  tile_mma<false, true>(Ai, Aj, acc);
  const int r0 = (threadIdx.x / 16) * 4, c0 = (threadIdx.x % 16) * 4;
  double* C = M + (size_t)i * TD * np + (size_t)j * TD;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int p = 0; p < 4; ++p) C[(size_t)(r0 + q) * np + c0 + p] -= acc[q][p];
}

// Inverse of every diagonal tile of L (lower triangular): column c of the
// inverse solves L_bb y = e_c; thread c of the block handles column c.
__global__ __launch_bounds__(256) void k_trtri_diag(const double* L, double* Li, int np) {
  __shared__ double T[TD][TD + 1], X[TD][TD + 1];
  const int b = blockIdx.x;
  load_tile(T, L, np, b, b);
  __syncthreads();
  const int c = threadIdx.x;
  if (c < TD) {
    for (int r = 0; r < TD; ++r) {
      double s = (r == c) ? 1.0 : 0.0;
      if (r >= c) {
        for (int l = c; l < r; ++l) s -= T[r][l] * X[l][c];
        s /= T[r][r];
      }
      X[r][c] = s;
    }
  }
  __syncthreads();
  double* D = Li + (size_t)b * TD * np + (size_t)b * TD;
  for (int e = threadIdx.x; e < TD * TD; e += blockDim.x) {
    const int r = e / TD, cc = e % TD;
    D[(size_t)r * np + cc] = X[r][cc];
  }
}

// Block row i of L^{-1}: for j < i (one block each),
//   Linv_ij = -Linv_ii * sum_{k=j}^{i-1} L_ik Linv_kj.
__global__ __launch_bounds__(256) void k_trtri_row(const double* L, double* Li, int np, int i) {
  __shared__ double S1[TD][TD + 1], S2[TD][TD + 1];
  const int j = blockIdx.x;
  double acc[4][4] = {};
  for (int k = j; k < i; ++k) {
    load_tile(S1, L, np, i, k);
    load_tile(S2, Li, np, k, j);
    __syncthreads();
    tile_mma<false, false>(S1, S2, acc);
    __syncthreads();
  }
  const int r0 = (threadIdx.x / 16) * 4, c0 = (threadIdx.x % 16) * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int p = 0; p < 4; ++p) S2[r0 + q][c0 + p] = acc[q][p];
  load_tile(S1, Li, np, i, i);
  __syncthreads();
  double out[4][4] = {};
  tile_mma<false, false>(S1, S2, out);
  double* D = Li + (size_t)i * TD * np + (size_t)j * TD;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int p = 0; p < 4; ++p) D[(size_t)(r0 + q) * np + c0 + p] = -out[q][p];
}

// X = Linv^T Linv: X_ij = sum_{k = i}^{nb-1} Linv_ki^T Linv_kj for i >= j,
// written to both X_ij and X_ji (2-D grid; blocks above the diagonal return).
__global__ __launch_bounds__(256) void k_lauum(const double* Li, double* X, int np) {
  const int nb = np / TD;
  const int i = blockIdx.y, j = blockIdx.x;
  if (j > i) return;
  __shared__ double S1[TD][TD + 1], S2[TD][TD + 1];
  double acc[4][4] = {};
  for (int k = i; k < nb; ++k) {
    load_tile(S1, Li, np, k, i);
    load_tile(S2, Li, np, k, j);
    __syncthreads();
    tile_mma<true, false>(S1, S2, acc);
    __syncthreads();
  }
  const int r0 = (threadIdx.x / 16) * 4, c0 = (threadIdx.x % 16) * 4;
  double* D = X + (size_t)i * TD * np + (size_t)j * TD;
  double* E = X + (size_t)j * TD * np + (size_t)i * TD;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      D[(size_t)(r0 + q) * np + c0 + p] = acc[q][p];
      if (i != j) E[(size_t)(c0 + p) * np + r0 + q] = acc[q][p];
    }
}

// Dense copy of the coarsest CSR matrix into the padded array (zeroed before),
// identity on the padding diagonal.
__global__ __launch_bounds__(256) void k_csr_to_padded(int n, int np, const int* __restrict__ rp,
                                                       const int* __restrict__ ci, const double* __restrict__ v,
                                                       double* __restrict__ M) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
    if (i < n) {
      for (int e = rp[i]; e < rp[i + 1]; ++e) M[(size_t)i * np + ci[e]] += v[e];
    } else {
      M[(size_t)i * np + i] = 1.0;
    }
  }
}

}  // namespace mvamg
