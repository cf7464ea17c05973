// Host side of the small-problem batch path (mini_kernels.hpp): the layout of
// every problem's hierarchy in its smoother order, and the coarsest inverse.
// Included by mvamg_lib.hip inside its anonymous namespace.

// Dense inverse of the s.p.d. n x n matrix of level C (row-major), from its
// Cholesky factor: column j of the inverse solves L L^T y = e_j.
std::vector<double> dense_spd_inverse(const HostLevel& C) {
  const int n = C.n;
  std::vector<double> M((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int e = C.rp[i]; e < C.rp[i + 1]; ++e) M[(size_t)i * n + C.ci[e]] += C.v[e];
  for (int j = 0; j < n; ++j) {
    double d = M[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= M[(size_t)j * n + k] * M[(size_t)j * n + k];
    if (!(d > 0.0)) throw Error(MVAMG_ERR_NOT_SPD, "coarsest matrix is not positive definite (Cholesky pivot <= 0)");
    d = std::sqrt(d);
    M[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = M[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= M[(size_t)i * n + k] * M[(size_t)j * n + k];
      M[(size_t)i * n + j] = s / d;
    }
  }
  std::vector<double> inv((size_t)n * n), y(n);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) {  // L y = e_j
      double s = (i == j) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= M[(size_t)i * n + k] * y[k];
      y[i] = s / M[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {  // L^T x = y
      double s = y[i];
      for (int k = i + 1; k < n; ++k) s -= M[(size_t)k * n + i] * y[k];
      y[i] = s / M[(size_t)i * n + i];
    }
    // column j of the inverse, stored contiguously: inv[j n + i] = (A^-1)_ij
    for (int i = 0; i < n; ++i) inv[(size_t)j * n + i] = y[i];
  }
  return inv;
}

constexpr int kMiniMaxCoarsest = 2048;

struct MiniBuild {
  std::vector<MiniProb> probs;
  std::vector<MiniLevel> levs;
  std::vector<int> ints;
  std::vector<double> dbls;
  int64_t work = 0;  // doubles of work space
};

// Appends problem H (rows row0 .. row0 + n - 1 of the batch vectors).
void mini_add(MiniBuild& B, const HostHier& H, int64_t row0) {
  if (H.nl < 2 || H.nl > kMiniMaxLevels) throw Error(MVAMG_ERR_ARG, "small-problem path: 2 to 16 levels");
  const HostLevel& Cst = H.lv[H.nl - 1];
  if (Cst.n > kMiniMaxCoarsest) throw Error(MVAMG_ERR_ARG, "small-problem path: coarsest level above 2048 rows");
  auto put_i = [&](const std::vector<int>& v) {
    const int64_t off = (int64_t)B.ints.size();
    B.ints.insert(B.ints.end(), v.begin(), v.end());
    return off;
  };
  auto put_d = [&](const std::vector<double>& v) {
    const int64_t off = (int64_t)B.dbls.size();
    B.dbls.insert(B.dbls.end(), v.begin(), v.end());
    return off;
  };
  auto take_w = [&](int64_t n) {
    const int64_t off = B.work;
    B.work += n;
    return off;
  };
  // smoother order of every level (identity on the coarsest) and its inverse
  std::vector<std::vector<int>> perm(H.nl), iperm(H.nl);
  for (int l = 0; l < H.nl; ++l) {
    const HostLevel& L = H.lv[l];
    if (l + 1 < H.nl) {
      perm[l] = L.order;
    } else {
      perm[l].resize(L.n);
      for (int i = 0; i < L.n; ++i) perm[l][i] = i;
    }
    iperm[l].assign(L.n, -1);
    for (int i = 0; i < L.n; ++i) iperm[l][perm[l][i]] = i;
  }
  MiniProb P{};
  P.nl = H.nl;
  P.lev0 = (int)B.levs.size();
  P.n = H.lv[0].n;
  P.row0 = row0;
  P.perm0 = put_i(perm[0]);
  for (int l = 0; l < H.nl; ++l) {
    const HostLevel& L = H.lv[l];
    MiniLevel M{};
    M.n = L.n;
    // CSR in smoother order, entries of a row in the file's order
    std::vector<int> rp(L.n + 1, 0), ci;
    std::vector<double> va, dg(L.n, 0.0), dl(L.n, 0.0);
    ci.reserve(L.ci.size());
    va.reserve(L.v.size());
    for (int i = 0; i < L.n; ++i) {
      const int f = perm[l][i];
      for (int e = L.rp[f]; e < L.rp[f + 1]; ++e) {
        const int j = iperm[l][L.ci[e]];
        ci.push_back(j);
        va.push_back(L.v[e]);
        if (j == i) dg[i] += L.v[e];
        dl[i] += std::fabs(L.v[e]);
      }
      rp[i + 1] = (int)ci.size();
      if (l + 1 < H.nl && !(dg[i] > 0.0)) throw Error(MVAMG_ERR_ARG, "non-positive diagonal");
    }
    M.rp = put_i(rp);
    M.ci = put_i(ci);
    M.va = put_d(va);
    M.dg = put_d(dg);
    M.dl = put_d(dl);
    M.r = take_w(L.n);
    M.x = take_w(L.n);
    M.s = take_w(L.n);
    if (l + 1 < H.nl) {
      M.ns = (int)L.sptr.size() - 1;
      M.sgrp = put_i(L.sptr);
      M.gptr = put_i(L.gptr);
      M.nagg = (int)L.aptr.size() - 1;
      std::vector<int> arows(L.arows.size()), cdof;
      for (size_t q = 0; q < L.arows.size(); ++q) arows[q] = iperm[l][L.arows[q]];
      for (int c = 0; c < H.lv[l + 1].n; ++c) cdof.push_back(iperm[l + 1][c]);
      M.aptr = put_i(L.aptr);
      M.arows = put_i(arows);
      M.cptr = put_i(L.coff);
      M.cdof = put_i(cdof);
      M.uoff = put_i(L.uoff);
      M.U = put_d(L.U);
    }
    B.levs.push_back(M);
  }
  P.ainv = put_d(dense_spd_inverse(Cst));
  P.cr = take_w(P.n);
  P.cz = take_w(P.n);
  P.cp = take_w(P.n);
  P.cq = take_w(P.n);
  P.cx = take_w(P.n);
  B.probs.push_back(P);
}
