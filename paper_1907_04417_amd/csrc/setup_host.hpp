// Host side of the numeric level setup (Section 4): argument checks, the
// coarse pattern of the Galerkin product (which aggregates are coupled), and
// the launches of setup_kernels.hpp.  Included by mvamg_lib.hip inside its
// anonymous namespace.

// LDS of one bases workgroup: the n_a x m block
constexpr size_t kSetupLdsMax = 64 * 1024;

void setup_bases(int m, int nagg, int max_na, const int* aptr, const int* arows, const double* W, double tol,
                 int n_level, int* k, double* U, double* dropped, int* flag, hipStream_t st) {
  if (m < 1 || m > kSvdMaxM) throw Error(MVAMG_ERR_ARG, "between 1 and 16 smooth vectors");
  if (nagg < 1 || max_na < 1 || n_level < 1) throw Error(MVAMG_ERR_ARG, "empty level");
  const size_t lds = (size_t)max_na * m * sizeof(double);
  if (lds > kSetupLdsMax) throw Error(MVAMG_ERR_ARG, "aggregate too large for the bases kernel (n_a m > 8192)");
  if (!(tol >= 0.0)) throw Error(MVAMG_ERR_ARG, "negative TOL");
  k_fill<int><<<1, kBlock, 0, st>>>(1, 0, flag);
  k_setup_bases<<<nagg, 64, lds, st>>>(m, nagg, aptr, arows, W, tol / (double)n_level, k, U, dropped, flag);
  LAUNCHCHECK("setup_bases");
  int hflag = 0;
  HIPCHECK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  if (hflag) throw Error(MVAMG_ERR_ARG, "an aggregate whose smooth vectors are all zero");
}

// The coarse pattern of P^T A P: the rows of aggregate a (coarse dofs
// coff[a] .. coff[a] + k_a - 1) couple to every dof of every aggregate that a
// row of a couples to in A; columns sorted.  Fills agg (n: aggregate of each
// fine row), loc (n: the row's place among its aggregate's members), coff
// (nagg + 1), cagg (nc: aggregate of each coarse dof) and, when crp is not
// null, crp (nc + 1) and ccol (nnz).  Returns the coarse nonzero count.
int64_t galerkin_pattern(int n, const int* rowptr, const int* col, int nagg, const int* aptr, const int* arows,
                         const int* k, int* agg, int* loc, int* coff, int* cagg, int* crp, int* ccol) {
  if (n < 1 || nagg < 1) throw Error(MVAMG_ERR_ARG, "empty level");
  if (aptr[0] != 0 || aptr[nagg] != n) throw Error(MVAMG_ERR_ARG, "aggregates do not cover the level");
  for (int i = 0; i < n; ++i) agg[i] = -1;
  coff[0] = 0;
  for (int a = 0; a < nagg; ++a) {
    if (aptr[a + 1] <= aptr[a]) throw Error(MVAMG_ERR_ARG, "empty aggregate");
    if (k[a] < 1 || k[a] > aptr[a + 1] - aptr[a]) throw Error(MVAMG_ERR_ARG, "basis width out of range");
    for (int q = aptr[a]; q < aptr[a + 1]; ++q) {
      const int i = arows[q];
      if (i < 0 || i >= n || agg[i] >= 0) throw Error(MVAMG_ERR_ARG, "aggregates are not a partition of the rows");
      agg[i] = a;
      loc[i] = q - aptr[a];
    }
    coff[a + 1] = coff[a] + k[a];
  }
  for (int a = 0; a < nagg; ++a)
    for (int c = coff[a]; c < coff[a + 1]; ++c) cagg[c] = a;
  std::vector<int> mark(nagg, -1), nb;
  int64_t nnz = 0;
  if (crp) crp[0] = 0;
  for (int a = 0; a < nagg; ++a) {
    nb.clear();
    for (int q = aptr[a]; q < aptr[a + 1]; ++q) {
      const int i = arows[q];
      for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const int j = col[e];
        if (j < 0 || j >= n) throw Error(MVAMG_ERR_ARG, "column index out of range");
        const int b = agg[j];
        if (mark[b] != a) {
          mark[b] = a;
          nb.push_back(b);
        }
      }
    }
    std::sort(nb.begin(), nb.end());
    int64_t len = 0;
    for (int b : nb) len += k[b];
    if (len > INT_MAX) throw Error(MVAMG_ERR_ARG, "coarse row too long");
    for (int l = 0; l < k[a]; ++l) {
      const int I = coff[a] + l;
      if (crp) {
        if (nnz + len > INT_MAX) throw Error(MVAMG_ERR_ARG, "coarse matrix too large for 32-bit offsets");
        int64_t p = nnz;
        for (int b : nb)
          for (int mm = 0; mm < k[b]; ++mm) ccol[p++] = coff[b] + mm;
        crp[I + 1] = (int)(nnz + len);
      }
      nnz += len;
    }
  }
  return nnz;
}
