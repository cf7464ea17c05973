// Host setup of the single-hierarchy multiple-vector aggregation-based AMG.
//
// This is the input generator of the solve phase: it runs on the CPU, is not
// timed, and writes the hierarchy to a file that both the GPU library and the
// CPU oracle read.  It implements, in order:
//
//   * the bootstrap of Section 2 (Algorithm 1): stage r builds a new
//     aggregation AMG operator B_r from the smooth vector w_{r-1} and tests
//     the symmetrized multiplicative composite
//         (I - B_1 A)...(I - B_r A)(I - B_r A)...(I - B_1 A)
//     nu times on a random vector (Section 5, items (i)-(ii)); the last iterate,
//     A-normalised, is the next smooth vector w_r;
//   * coarsening based on compatible weighted matching (Section 3): pairwise
//     aggregates from an approximate maximum-product matching of the graph of
//     A with edge weights derived from eq. (3.1)-(3.3); piecewise-constant
//     prolongator P_c of eq. (3.2); two matching steps per level ("double
//     pairwise"), A_c = P^T A P;
//   * the multiple-vector hierarchy of Section 4: aggregates composed from
//     `compose` consecutive levels of one bootstrap hierarchy (eq. 4.1-4.2, the
//     Q map of Section 4.1 for coarse levels), per-aggregate SVD of the
//     restricted smooth vectors (eq. 4.3) truncated at
//     TOL * size(a)/size(A) (Section 5), block-diagonal orthonormal P and
//     Galerkin coarse matrices, smooth vectors projected level by level;
//   * a direct solve on the coarsest level of every bootstrap hierarchy: a
//     dense Cholesky factor, or a sparse one (minimum-degree order) where a
//     stalled coarsening left that level large;
//   * the Gauss-Seidel order of every non-coarsest level: a greedy first-fit
//     colouring of groups of rows (single rows on the finest level, the k_a
//     coarse dofs of one aggregate on coarser levels), groups listed colour by
//     colour.
//
// All parallel loops are written so that results do not depend on the number
// of threads (fixed-size chunks for reductions, per-row independent work).

#include <algorithm>
#include <random>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include <omp.h>

namespace {

thread_local std::string g_err;

struct Csr {
  int n = 0;
  std::vector<int> rp, ci;
  std::vector<double> v;
  int64_t nnz() const { return rp.empty() ? 0 : rp[n]; }
};

struct Colouring {
  int ncol = 0;
  std::vector<int> cptr, crows;
};

// Piecewise-constant pairwise / composite map: fine node i -> coarse agg[i],
// with prolongator value p[i] (one nonzero per fine row).
struct PcMap {
  int nc = 0;
  std::vector<int> agg;
  std::vector<double> p;
};

struct Fail {
  std::string msg;
};

[[noreturn]] void fail(const std::string& m) { throw Fail{m}; }

constexpr int kChunk = 8192;

double dot(const double* a, const double* b, int n) {
  const int nch = (n + kChunk - 1) / kChunk;
  std::vector<double> part(nch);
#pragma omp parallel for schedule(static)
  for (int c = 0; c < nch; ++c) {
    const int lo = c * kChunk, hi = std::min(n, lo + kChunk);
    double s = 0.0;
    for (int i = lo; i < hi; ++i) s += a[i] * b[i];
    part[c] = s;
  }
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += part[c];
  return s;
}

void spmv(const Csr& A, const double* x, double* y) {
#pragma omp parallel for schedule(static, 1024)
  for (int i = 0; i < A.n; ++i) {
    double s = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) s += A.v[k] * x[A.ci[k]];
    y[i] = s;
  }
}

std::vector<double> diag_of(const Csr& A) {
  std::vector<double> d(A.n, 0.0);
  bool bad = false;
#pragma omp parallel for schedule(static, 4096) reduction(|| : bad)
  for (int i = 0; i < A.n; ++i) {
    bool found = false;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] == i) {
        d[i] = A.v[k];
        found = true;
      }
    if (!found || !(d[i] > 0.0)) bad = true;
  }
  if (bad) fail("matrix has a missing or non-positive diagonal entry (not s.p.d.)");
  return d;
}

// Greedy first-fit colouring in natural row order.
Colouring greedy_colour(const Csr& A) {
  Colouring C;
  std::vector<int> colour(A.n, -1);
  std::vector<int> forbid;
  for (int i = 0; i < A.n; ++i) {
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int j = A.ci[k];
      if (j != i && colour[j] >= 0) forbid[colour[j]] = i;
    }
    int c = 0;
    while (c < (int)forbid.size() && forbid[c] == i) ++c;
    if (c == (int)forbid.size()) forbid.push_back(-1);
    colour[i] = c;
  }
  C.ncol = (int)forbid.size();
  C.cptr.assign(C.ncol + 1, 0);
  for (int i = 0; i < A.n; ++i) C.cptr[colour[i] + 1]++;
  for (int c = 0; c < C.ncol; ++c) C.cptr[c + 1] += C.cptr[c];
  C.crows.resize(A.n);
  std::vector<int> pos(C.cptr.begin(), C.cptr.end() - 1);
  for (int i = 0; i < A.n; ++i) C.crows[pos[colour[i]]++] = i;
  return C;
}

// One multicolour Gauss-Seidel sweep: rows of colour c are updated together
// (they are not coupled), colours taken in increasing (forward) or decreasing
// (backward) order.
void gs_sweep(const Csr& A, const std::vector<double>& d, const Colouring& C,
              const double* r, double* x, bool forward) {
  for (int cc = 0; cc < C.ncol; ++cc) {
    const int c = forward ? cc : C.ncol - 1 - cc;
#pragma omp parallel for schedule(static, 512)
    for (int q = C.cptr[c]; q < C.cptr[c + 1]; ++q) {
      const int i = C.crows[q];
      double s = r[i];
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
        if (A.ci[k] != i) s -= A.v[k] * x[A.ci[k]];
      x[i] = s / d[i];
    }
  }
}

// Lowers the number of colours of a proper colouring of the graph (gp, gi)
// (CSR, no self loops) by tabu search -- TabuCol (Hertz and de Werra, 1987)
// with the tabu tenure of Galinier and Hao (1999).  For a target of k colours
// the vertices coloured k or higher take their least-conflicting colour below
// k; then, repeatedly, the move of one conflicting vertex to another colour
// that lowers the number of monochromatic edges most is made (ties broken by a
// fixed-seed generator, moves back to a recently left colour forbidden for
// 10 + U{0..9} + 0.6 * conflicts moves unless they reach a new best).  A target
// reached without conflicts replaces the colouring and the next lower one is
// tried; the search stops at the first target not reached within `budget`
// move evaluations.  Deterministic for a given graph and start.
int reduce_colours(const std::vector<int>& gp, const std::vector<int>& gi, std::vector<int>& col, int ncol,
                   int64_t budget) {
  const int n = (int)col.size();
  std::mt19937 rng(20260101u);
  for (int k = ncol - 1; k >= 2; --k) {
    std::vector<int> c2 = col;
    std::vector<int> cnt(k);
    for (int g = 0; g < n; ++g)
      if (c2[g] >= k) c2[g] = -1;
    for (int g = 0; g < n; ++g)
      if (c2[g] < 0) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int e = gp[g]; e < gp[g + 1]; ++e)
          if (c2[gi[e]] >= 0) cnt[c2[gi[e]]]++;
        c2[g] = (int)(std::min_element(cnt.begin(), cnt.end()) - cnt.begin());
      }
    std::vector<int> gamma((size_t)n * k, 0);  // neighbours of g with colour c
    for (int g = 0; g < n; ++g)
      for (int e = gp[g]; e < gp[g + 1]; ++e) gamma[(size_t)g * k + c2[gi[e]]]++;
    std::vector<int> cv, cpos(n, -1);  // conflicting vertices
    auto track = [&](int g) {
      const bool in = gamma[(size_t)g * k + c2[g]] > 0;
      if (in && cpos[g] < 0) {
        cpos[g] = (int)cv.size();
        cv.push_back(g);
      } else if (!in && cpos[g] >= 0) {
        const int last = cv.back();
        cv[cpos[g]] = last;
        cpos[last] = cpos[g];
        cv.pop_back();
        cpos[g] = -1;
      }
    };
    int64_t conf = 0;
    for (int g = 0; g < n; ++g) {
      conf += gamma[(size_t)g * k + c2[g]];
      track(g);
    }
    conf /= 2;
    std::vector<int64_t> tabu((size_t)n * k, 0);
    int64_t it = 0, evals = 0, best = conf;
    while (conf > 0 && evals < budget) {
      ++it;
      int bg = -1, bc = -1, ties = 0;
      int64_t bd = INT64_MAX;
      for (const int g : cv) {
        const int* gm = gamma.data() + (size_t)g * k;
        const int cg = c2[g];
        for (int c = 0; c < k; ++c) {
          if (c == cg) continue;
          ++evals;
          const int64_t d = (int64_t)gm[c] - gm[cg];
          if (tabu[(size_t)g * k + c] > it && !(conf + d < best)) continue;
          if (d < bd) {
            bd = d;
            bg = g;
            bc = c;
            ties = 1;
          } else if (d == bd && rng() % (uint32_t)(++ties) == 0) {
            bg = g;
            bc = c;
          }
        }
      }
      if (bg < 0) break;
      const int old = c2[bg];
      c2[bg] = bc;
      conf += bd;
      for (int e = gp[bg]; e < gp[bg + 1]; ++e) {
        const int h = gi[e];
        gamma[(size_t)h * k + old]--;
        gamma[(size_t)h * k + bc]++;
        track(h);
      }
      track(bg);
      tabu[(size_t)bg * k + old] = it + 10 + (int64_t)(rng() % 10u) + (int64_t)(0.6 * (double)conf);
      best = std::min(best, conf);
    }
    if (conf > 0) break;
    col.swap(c2);
    ncol = k;
  }
  return ncol;
}

// Size of a clique found greedily in the graph (gp, gi) (CSR, sorted
// neighbour lists, no self loops): from every vertex, its neighbours are added
// in order when adjacent to all vertices taken so far.  A lower bound on the
// chromatic number: a colouring with that many colours cannot be improved.
int greedy_clique(const std::vector<int>& gp, const std::vector<int>& gi) {
  const int n = (int)gp.size() - 1;
  auto adjacent = [&](int a, int b) { return std::binary_search(gi.begin() + gp[a], gi.begin() + gp[a + 1], b); };
  int best = n > 0 ? 1 : 0;
  std::vector<int> c;
  for (int v = 0; v < n; ++v) {
    c.assign(1, v);
    for (int e = gp[v]; e < gp[v + 1]; ++e) {
      const int u = gi[e];
      bool all = true;
      for (size_t i = 1; i < c.size() && all; ++i) all = adjacent(u, c[i]);
      if (all) c.push_back(u);
    }
    best = std::max(best, (int)c.size());
  }
  return best;
}

// Smoother ordering of a multi-vector level.  Rows are split into groups of
// consecutive indices (gstart); groups are coloured greedily (first fit, in
// natural group order) on the graph in which two groups are adjacent when A
// couples any of their rows, and the colour count is then lowered by
// reduce_colours (fewer colours: fewer stages, each a kernel launch).  The Gauss-Seidel order O lists the groups colour
// by colour ("stages"), the rows of a group in increasing index.  Groups of one
// stage are not coupled, so they can be relaxed simultaneously; the rows of a
// group are relaxed one after the other.
struct GsOrder {
  std::vector<int> order, gptr, sptr;
};

GsOrder group_order(const Csr& A, const std::vector<int>& gstart) {
  const int G = (int)gstart.size() - 1;
  std::vector<int> grp(A.n);
  for (int g = 0; g < G; ++g)
    for (int i = gstart[g]; i < gstart[g + 1]; ++i) grp[i] = g;
  std::vector<int> gcol(G, -1), forbid;
  for (int g = 0; g < G; ++g) {
    for (int i = gstart[g]; i < gstart[g + 1]; ++i)
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int h = grp[A.ci[k]];
        if (h != g && gcol[h] >= 0) forbid[gcol[h]] = g;
      }
    int c = 0;
    while (c < (int)forbid.size() && forbid[c] == g) ++c;
    if (c == (int)forbid.size()) forbid.push_back(-1);
    gcol[g] = c;
  }
  int ncol = (int)forbid.size();
  if (ncol > 2) {
    std::vector<int> gp(G + 1, 0), gi, mark(G, -1);
    for (int g = 0; g < G; ++g) {
      for (int i = gstart[g]; i < gstart[g + 1]; ++i)
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
          const int h = grp[A.ci[k]];
          if (h != g && mark[h] != g) {
            mark[h] = g;
            gi.push_back(h);
          }
        }
      gp[g + 1] = (int)gi.size();
    }
    for (int g = 0; g < G; ++g) std::sort(gi.begin() + gp[g], gi.begin() + gp[g + 1]);
    if (greedy_clique(gp, gi) < ncol)
      ncol = reduce_colours(gp, gi, gcol, ncol, std::min<int64_t>(100 * (int64_t)gi.size() + 10000000, 400000000));
  }
  GsOrder O;
  O.sptr.assign(ncol + 1, 0);
  for (int g = 0; g < G; ++g) O.sptr[gcol[g] + 1]++;
  for (int c = 0; c < ncol; ++c) O.sptr[c + 1] += O.sptr[c];
  std::vector<int> gs(G), pos(O.sptr.begin(), O.sptr.end() - 1);
  for (int g = 0; g < G; ++g) gs[pos[gcol[g]]++] = g;
  O.gptr.assign(G + 1, 0);
  O.order.reserve(A.n);
  for (int t = 0; t < G; ++t) {
    const int g = gs[t];
    for (int i = gstart[g]; i < gstart[g + 1]; ++i) O.order.push_back(i);
    O.gptr[t + 1] = (int)O.order.size();
  }
  return O;
}

// Make stored values bitwise symmetric: v_ij = v_ji = (v_ij + v_ji)/2.
// Requires a structurally symmetric matrix with sorted column indices.
void symmetrize(Csr& A) {
  bool bad = false;
#pragma omp parallel for schedule(dynamic, 256) reduction(|| : bad)
  for (int i = 0; i < A.n; ++i) {
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int j = A.ci[k];
      if (j <= i) continue;
      const int* b = A.ci.data() + A.rp[j];
      const int* e = A.ci.data() + A.rp[j + 1];
      const int* f = std::lower_bound(b, e, i);
      if (f == e || *f != i) {
        bad = true;
        continue;
      }
      const int64_t kt = f - A.ci.data();
      const double m = 0.5 * (A.v[k] + A.v[kt]);
      A.v[k] = m;
      A.v[kt] = m;
    }
  }
  if (bad) fail("Galerkin product is not structurally symmetric");
}

// Edge weight of the compatible weighted matching (Section 3): the diagonal
// entry of A_f = P_f^T A P_f belonging to the pair e = {i, j}, i.e. the
// quadratic form (w_e^perp)^T A_ee w_e^perp with w_e^perp from eq. (3.1):
//     c_ij = 1 - 2 a_ij w_i w_j / (a_ii w_i^2 + a_jj w_j^2).
// Evaluated with the lower index first so that c_ij == c_ji bitwise.
inline double edge_weight(double aij, double dlo, double dhi, double wlo, double whi) {
  const double den = dlo * wlo * wlo + dhi * whi * whi;
  if (den == 0.0) return 1.0;
  return 1.0 - 2.0 * aij * wlo * whi / den;
}

// Strict total order on edges: larger weight first, then smaller (lo, hi).
inline bool edge_better(double c1, int lo1, int hi1, double c2, int lo2, int hi2) {
  if (c1 != c2) return c1 > c2;
  if (lo1 != lo2) return lo1 < lo2;
  return hi1 < hi2;
}

// Approximate maximum-weight matching by locally dominant edges
// (Preis 1999; Manne & Bisseling 2007): every unmatched vertex points to its
// best available neighbour; mutually pointing pairs are matched; repeat.
// With a strict total order on edges this equals the greedy 1/2-approximation
// and does not depend on the thread count.  Only edges of positive weight
// are eligible.
std::vector<int> match_locally_dominant(const Csr& A, const std::vector<double>& d,
                                        const std::vector<double>& w) {
  const int n = A.n;
  std::vector<double> cw(A.nnz());
#pragma omp parallel for schedule(static, 1024)
  for (int i = 0; i < n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int j = A.ci[k];
      if (j == i) {
        cw[k] = -1.0;
        continue;
      }
      const int lo = std::min(i, j), hi = std::max(i, j);
      cw[k] = edge_weight(A.v[k], d[lo], d[hi], w[lo], w[hi]);
    }
  std::vector<int> mate(n, -1), cand(n, -1);
  for (int round = 0; round < 1000000; ++round) {
#pragma omp parallel for schedule(static, 1024)
    for (int i = 0; i < n; ++i) {
      cand[i] = -1;
      if (mate[i] != -1) continue;
      int best = -1;
      double bw = 0.0;
      int blo = 0, bhi = 0;
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int j = A.ci[k];
        if (j == i || mate[j] != -1) continue;
        const double c = cw[k];
        if (!(c > 0.0)) continue;
        const int lo = std::min(i, j), hi = std::max(i, j);
        if (best < 0 || edge_better(c, lo, hi, bw, blo, bhi)) {
          best = j;
          bw = c;
          blo = lo;
          bhi = hi;
        }
      }
      cand[i] = best;
    }
    int64_t nm = 0;
#pragma omp parallel for schedule(static, 1024) reduction(+ : nm)
    for (int i = 0; i < n; ++i) {
      const int j = cand[i];
      if (mate[i] == -1 && j >= 0 && cand[j] == i) {
        mate[i] = j;
        ++nm;
      }
    }
    if (nm == 0) break;
  }
  return mate;
}

// One pairwise aggregation step: matching, coarse numbering in natural order
// of the smallest member, and the values of P_c (eq. 3.2): w_e for a pair,
// w_k/|w_k| for an unmatched node (+1 when w_k = 0).
PcMap pairwise(const Csr& A, const std::vector<double>& d, const std::vector<double>& w) {
  const int n = A.n;
  std::vector<int> mate = match_locally_dominant(A, d, w);
  PcMap P;
  P.agg.assign(n, -1);
  P.p.assign(n, 0.0);
  int nc = 0;
  for (int i = 0; i < n; ++i) {
    if (P.agg[i] >= 0) continue;
    P.agg[i] = nc;
    const int j = mate[i];
    if (j >= 0) {
      P.agg[j] = nc;
      const double nrm = std::sqrt(w[i] * w[i] + w[j] * w[j]);
      if (nrm > 0.0) {
        P.p[i] = w[i] / nrm;
        P.p[j] = w[j] / nrm;
      } else {
        P.p[i] = P.p[j] = 1.0 / std::sqrt(2.0);
      }
    } else {
      P.p[i] = (w[i] < 0.0) ? -1.0 : 1.0;
    }
    ++nc;
  }
  P.nc = nc;
  return P;
}

// Members of each coarse node, in increasing fine index.
void members(const std::vector<int>& agg, int nc, std::vector<int>& mptr, std::vector<int>& mem) {
  mptr.assign(nc + 1, 0);
  for (int a : agg) mptr[a + 1]++;
  for (int c = 0; c < nc; ++c) mptr[c + 1] += mptr[c];
  mem.resize(agg.size());
  std::vector<int> pos(mptr.begin(), mptr.end() - 1);
  for (int i = 0; i < (int)agg.size(); ++i) mem[pos[agg[i]]++] = i;
}

Csr assemble(int n, std::vector<std::vector<int>>& cols, std::vector<std::vector<double>>& vals) {
  Csr A;
  A.n = n;
  A.rp.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    if ((int64_t)A.rp[i] + (int64_t)cols[i].size() > std::numeric_limits<int>::max())
      fail("coarse matrix exceeds 2^31 nonzeros");
    A.rp[i + 1] = A.rp[i] + (int)cols[i].size();
  }
  A.ci.resize(A.rp[n]);
  A.v.resize(A.rp[n]);
#pragma omp parallel for schedule(static, 256)
  for (int i = 0; i < n; ++i) {
    std::copy(cols[i].begin(), cols[i].end(), A.ci.begin() + A.rp[i]);
    std::copy(vals[i].begin(), vals[i].end(), A.v.begin() + A.rp[i]);
    std::vector<int>().swap(cols[i]);
    std::vector<double>().swap(vals[i]);
  }
  return A;
}

// Galerkin product P^T A P for a piecewise-constant P (one value per fine row).
Csr galerkin_pc(const Csr& A, const PcMap& P) {
  const int nc = P.nc;
  std::vector<int> mptr, mem;
  members(P.agg, nc, mptr, mem);
  std::vector<std::vector<int>> cols(nc);
  std::vector<std::vector<double>> vals(nc);
#pragma omp parallel
  {
    std::vector<int> mark(nc, -1);
    std::vector<std::pair<int, double>> row;
#pragma omp for schedule(dynamic, 256)
    for (int I = 0; I < nc; ++I) {
      row.clear();
      for (int q = mptr[I]; q < mptr[I + 1]; ++q) {
        const int i = mem[q];
        const double pi = P.p[i];
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
          const int j = A.ci[k];
          const int J = P.agg[j];
          const double val = pi * A.v[k] * P.p[j];
          if (mark[J] < 0) {
            mark[J] = (int)row.size();
            row.push_back({J, val});
          } else {
            row[mark[J]].second += val;
          }
        }
      }
      for (auto& e : row) mark[e.first] = -1;
      std::sort(row.begin(), row.end(),
                [](const std::pair<int, double>& a, const std::pair<int, double>& b) {
                  return a.first < b.first;
                });
      cols[I].resize(row.size());
      vals[I].resize(row.size());
      for (size_t t = 0; t < row.size(); ++t) {
        cols[I][t] = row[t].first;
        vals[I][t] = row[t].second;
      }
    }
  }
  Csr Ac = assemble(nc, cols, vals);
  symmetrize(Ac);
  return Ac;
}

std::vector<double> restrict_pc(const PcMap& P, const std::vector<double>& w) {
  std::vector<double> wc(P.nc, 0.0);
  for (size_t i = 0; i < w.size(); ++i) wc[P.agg[i]] += P.p[i] * w[i];
  return wc;
}

// Dense Cholesky A = L L^T (lower triangle, row-major n x n), in place.
void dense_cholesky(std::vector<double>& M, int n) {
  for (int j = 0; j < n; ++j) {
    double s = M[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= M[(size_t)j * n + k] * M[(size_t)j * n + k];
    if (!(s > 0.0)) fail("coarsest matrix is not positive definite");
    const double ljj = std::sqrt(s);
    M[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = M[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= M[(size_t)i * n + k] * M[(size_t)j * n + k];
      M[(size_t)i * n + j] = t / ljj;
    }
  }
}

void dense_cholesky_solve(const std::vector<double>& L, int n, const double* b, double* x) {
  std::vector<double> y(n);
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * y[k];
    y[i] = s / L[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * x[k];
    x[i] = s / L[(size_t)i * n + i];
  }
}

// Sparse Cholesky L L^T = A(perm, perm) of a coarsest level too large for the
// dense factor (a bootstrap hierarchy whose coarsening stalled).  The pivot
// order is minimum degree on the elimination graph (ties to the lower index):
// eliminating a vertex joins its remaining neighbours into a clique, and that
// neighbour set is the pattern of its column of L.  The graphs a stall leaves
// are star-like (many degree-1 vertices around a few hubs), which this order
// eliminates leaf first, with little fill.
struct SparseChol {
  int n = 0;
  std::vector<int> perm;       // perm[k]: row of A eliminated k-th
  std::vector<int64_t> lp;     // column k of L below the diagonal: li/lx[lp[k] .. lp[k + 1])
  std::vector<int> li;         // pivot positions, increasing within a column
  std::vector<double> lx, ld;  // off-diagonal values, diagonal of L
};

SparseChol sparse_cholesky(const Csr& A) {
  const int n = A.n;
  SparseChol F;
  F.n = n;
  std::vector<std::vector<int>> adj(n);  // uneliminated neighbours, sorted
  for (int i = 0; i < n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] != i) adj[i].push_back(A.ci[k]);
  std::vector<char> gone(n, 0);
  std::vector<std::pair<int, int>> heap;  // (degree, vertex), lazily updated
  auto cmp = [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a > b; };
  for (int i = 0; i < n; ++i) heap.push_back({(int)adj[i].size(), i});
  std::make_heap(heap.begin(), heap.end(), cmp);
  std::vector<std::vector<int>> pat(n);  // column patterns as vertices
  std::vector<int> merged;
  F.perm.reserve(n);
  while (!heap.empty()) {
    std::pop_heap(heap.begin(), heap.end(), cmp);
    const auto [deg, v] = heap.back();
    heap.pop_back();
    if (gone[v] || deg != (int)adj[v].size()) continue;  // stale entry
    gone[v] = 1;
    F.perm.push_back(v);
    const std::vector<int>& nb = adj[v];
    for (int u : nb) {
      merged.clear();
      std::set_union(adj[u].begin(), adj[u].end(), nb.begin(), nb.end(), std::back_inserter(merged));
      merged.erase(std::remove_if(merged.begin(), merged.end(), [&](int x) { return x == u || x == v; }),
                   merged.end());
      const bool changed = merged.size() != adj[u].size();
      adj[u].swap(merged);
      if (changed) {  // the entry with the old degree goes stale
        heap.push_back({(int)adj[u].size(), u});
        std::push_heap(heap.begin(), heap.end(), cmp);
      }
    }
    pat[v] = std::move(adj[v]);
    adj[v].clear();
  }
  if ((int)F.perm.size() != n) fail("sparse coarsest factor: ordering incomplete");
  std::vector<int> pos(n);
  for (int k = 0; k < n; ++k) pos[F.perm[k]] = k;
  F.lp.assign(n + 1, 0);
  for (int k = 0; k < n; ++k) F.lp[k + 1] = F.lp[k] + (int64_t)pat[F.perm[k]].size();
  F.li.resize(F.lp[n]);
  F.lx.assign(F.lp[n], 0.0);
  F.ld.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    int* c = F.li.data() + F.lp[k];
    int t = 0;
    for (int u : pat[F.perm[k]]) c[t++] = pos[u];
    std::sort(c, c + t);
  }
  pat.clear();
  // rows of L: for pivot j, the columns k < j with L(j, k) != 0 and where j sits in them
  std::vector<int64_t> rp(n + 1, 0);
  for (int64_t q = 0; q < F.lp[n]; ++q) rp[F.li[q] + 1]++;
  for (int j = 0; j < n; ++j) rp[j + 1] += rp[j];
  std::vector<int64_t> rq(F.lp[n]), fill(rp.begin(), rp.end() - 1);
  std::vector<int> rk(F.lp[n]);
  for (int k = 0; k < n; ++k)
    for (int64_t q = F.lp[k]; q < F.lp[k + 1]; ++q) {
      rk[fill[F.li[q]]] = k;
      rq[fill[F.li[q]]++] = q;
    }
  // left-looking numeric factorization with a dense work column
  std::vector<double> w(n, 0.0);
  for (int j = 0; j < n; ++j) {
    const int r = F.perm[j];
    for (int k = A.rp[r]; k < A.rp[r + 1]; ++k) {
      const int pj = pos[A.ci[k]];
      if (pj >= j) w[pj] += A.v[k];
    }
    for (int64_t t = rp[j]; t < rp[j + 1]; ++t) {
      const int64_t q = rq[t];  // L(j, k) at position q of column k
      const int k = rk[t];
      const double ljk = F.lx[q];
      for (int64_t e = q; e < F.lp[k + 1]; ++e) w[F.li[e]] -= F.lx[e] * ljk;
    }
    const double d = w[j];
    if (!(d > 0.0)) fail("coarsest matrix is not positive definite");
    const double ljj = std::sqrt(d);
    F.ld[j] = ljj;
    w[j] = 0.0;
    for (int64_t e = F.lp[j]; e < F.lp[j + 1]; ++e) {
      F.lx[e] = w[F.li[e]] / ljj;
      w[F.li[e]] = 0.0;
    }
  }
  return F;
}

void sparse_cholesky_solve(const SparseChol& F, const double* b, double* x) {
  const int n = F.n;
  std::vector<double> y(n);
  for (int k = 0; k < n; ++k) y[k] = b[F.perm[k]];
  for (int j = 0; j < n; ++j) {
    y[j] /= F.ld[j];
    for (int64_t e = F.lp[j]; e < F.lp[j + 1]; ++e) y[F.li[e]] -= F.lx[e] * y[j];
  }
  for (int j = n - 1; j >= 0; --j) {
    double s = y[j];
    for (int64_t e = F.lp[j]; e < F.lp[j + 1]; ++e) s -= F.lx[e] * y[F.li[e]];
    y[j] = s / F.ld[j];
  }
  for (int k = 0; k < n; ++k) x[F.perm[k]] = y[k];
}

std::vector<double> densify(const Csr& A) {
  std::vector<double> M((size_t)A.n * A.n, 0.0);
  for (int i = 0; i < A.n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) M[(size_t)i * A.n + A.ci[k]] += A.v[k];
  return M;
}

// ---------------------------------------------------------------- bootstrap

struct BLevel {
  Csr A;
  std::vector<double> d;
  Colouring C;
  PcMap P;  // to the next level (empty on the coarsest)
  std::vector<double> r, x, s;  // work vectors
  std::vector<double> c1, c2, v1, v2, rt;  // K-cycle: the inner iterations on this level
};

struct BHier {
  std::vector<BLevel> lv;
  std::vector<double> Lc;  // dense Cholesky factor of the coarsest matrix
  SparseChol Fc;           // sparse factor instead, above the dense limit
  bool sparse = false;
  bool stalled = false;    // coarsening stopped above the dense limit
  int ncoarse = 0;
};

struct Params {
  int nvec_max;         // maximum number of smooth vectors (including w_0 = 1)
  int nu;               // testing-phase iterations per stage
  double rho_des;       // desired convergence factor
  int maxstage;         // maximum number of bootstrap stages
  double tol_svd;       // TOL of the per-aggregate truncation
  int compose;          // bootstrap levels merged per multi-vector level
  int coarse_cap;       // a multi-vector level of at most this size is the coarsest
  int boot_coarse_min;  // bootstrap hierarchies stop coarsening at this size
  int hier_stage;       // bootstrap hierarchy to compose: -1 last, else index (0 = first)
  int store_w;          // store projected smooth vectors in the file
  int max_levels;       // cap on bootstrap hierarchy depth
  int fine_group;       // rows per smoother group on the finest level (1: point)
  int boot_dense_max;   // largest bootstrap coarsest level factored densely
  int coarsest_max;     // largest coarsest multiple-vector level
  int boot_kcycle;      // the testing phase applies B_r as K-cycles (else V-cycles)
};

// Builds B_r's hierarchy from the fine matrix and smooth vector w
// (coarsening based on compatible weighted matching, two matching steps per
// level).
BHier build_bootstrap_hierarchy(const Csr& A0, const std::vector<double>& w0, const Params& prm) {
  BHier H;
  H.lv.emplace_back();
  H.lv[0].A = A0;
  std::vector<double> w = w0;
  for (int l = 0;; ++l) {
    BLevel& L = H.lv[l];
    L.d = diag_of(L.A);
    const int n = L.A.n;
    bool coarsest = (n <= prm.boot_coarse_min) || (l + 1 >= prm.max_levels);
    PcMap comp;
    Csr A2;
    std::vector<double> w2;
    if (!coarsest) {
      PcMap P1 = pairwise(L.A, L.d, w);
      Csr A1 = galerkin_pc(L.A, P1);
      std::vector<double> w1 = restrict_pc(P1, w);
      std::vector<double> d1 = diag_of(A1);
      PcMap P2 = pairwise(A1, d1, w1);
      A2 = galerkin_pc(A1, P2);
      w2 = restrict_pc(P2, w1);
      comp.nc = P2.nc;
      comp.agg.resize(n);
      comp.p.resize(n);
      for (int i = 0; i < n; ++i) {
        comp.agg[i] = P2.agg[P1.agg[i]];
        comp.p[i] = P1.p[i] * P2.p[P1.agg[i]];
      }
      // A stalled coarsening (a step that keeps more than 95% of the rows)
      // ends the hierarchy.  Matching-based pairwise steps stall where the
      // graph has turned star-like: a vertex whose only neighbour is matched
      // elsewhere stays a singleton and stays a leaf of that neighbour's
      // aggregate, so each further step can match only around the hubs.
      if ((double)comp.nc > 0.95 * (double)n) {
        coarsest = true;
        H.stalled = n > prm.boot_dense_max;
      }
    }
    if (coarsest) {
      // a direct solve on the coarsest level (Section 5); dense up to
      // boot_dense_max rows, sparse above
      if (n <= prm.boot_dense_max) {
        H.Lc = densify(L.A);
        dense_cholesky(H.Lc, n);
      } else {
        H.Fc = sparse_cholesky(L.A);
        H.sparse = true;
      }
      H.ncoarse = n;
      L.r.assign(n, 0.0);
      L.x.assign(n, 0.0);
      break;
    }
    L.C = greedy_colour(L.A);
    L.P = std::move(comp);
    L.r.assign(n, 0.0);
    L.x.assign(n, 0.0);
    L.s.assign(n, 0.0);
    if (l > 0 && prm.boot_kcycle)
      for (auto* v : {&L.c1, &L.c2, &L.v1, &L.v2, &L.rt}) v->assign(n, 0.0);
    BLevel next;
    next.A = std::move(A2);
    H.lv.push_back(std::move(next));
    w = std::move(w2);
  }
  return H;
}

// x = B r for the bootstrap hierarchy H (symmetric V-cycle: forward GS
// pre-smoothing, backward GS post-smoothing, direct coarsest solve).
void bh_vcycle(BHier& H, int l, const double* r, double* x) {
  BLevel& L = H.lv[l];
  const int n = L.A.n;
  if (l + 1 == (int)H.lv.size()) {
    if (H.sparse)
      sparse_cholesky_solve(H.Fc, r, x);
    else
      dense_cholesky_solve(H.Lc, n, r, x);
    return;
  }
  std::fill(x, x + n, 0.0);
  gs_sweep(L.A, L.d, L.C, r, x, true);
  spmv(L.A, x, L.s.data());
#pragma omp parallel for schedule(static, 4096)
  for (int i = 0; i < n; ++i) L.s[i] = r[i] - L.s[i];
  BLevel& C = H.lv[l + 1];
  std::fill(C.r.begin(), C.r.end(), 0.0);
  for (int i = 0; i < n; ++i) C.r[L.P.agg[i]] += L.P.p[i] * L.s[i];
  bh_vcycle(H, l + 1, C.r.data(), C.x.data());
#pragma omp parallel for schedule(static, 4096)
  for (int i = 0; i < n; ++i) x[i] += L.P.p[i] * C.x[L.P.agg[i]];
  gs_sweep(L.A, L.d, L.C, r, x, false);
}

// x = B r with the K-cycle (nonlinear AMLI): as the V-cycle, except that the
// coarse correction of a level whose next level is not the coarsest is two
// flexible-CG iterations on A_c e = r_c, each preconditioned by the K-cycle
// of the next level (Section 5; Notay and Vassilevski's K-cycle).  With
// c1 = B_c r_c, c2 = B_c (r_c - (c1' r_c / c1' A_c c1) A_c c1), the result is
// the A_c-orthogonal projection of the error onto span{c1, c2}.
void bh_kcycle(BHier& H, int l, const double* r, double* x) {
  BLevel& L = H.lv[l];
  const int n = L.A.n;
  if (l + 1 == (int)H.lv.size()) {
    if (H.sparse)
      sparse_cholesky_solve(H.Fc, r, x);
    else
      dense_cholesky_solve(H.Lc, n, r, x);
    return;
  }
  std::fill(x, x + n, 0.0);
  gs_sweep(L.A, L.d, L.C, r, x, true);
  spmv(L.A, x, L.s.data());
#pragma omp parallel for schedule(static, 4096)
  for (int i = 0; i < n; ++i) L.s[i] = r[i] - L.s[i];
  BLevel& C = H.lv[l + 1];
  const int nc = C.A.n;
  std::fill(C.r.begin(), C.r.end(), 0.0);
  for (int i = 0; i < n; ++i) C.r[L.P.agg[i]] += L.P.p[i] * L.s[i];
  if (l + 2 == (int)H.lv.size()) {
    bh_kcycle(H, l + 1, C.r.data(), C.x.data());  // exact on the coarsest
  } else {
    bh_kcycle(H, l + 1, C.r.data(), C.c1.data());
    spmv(C.A, C.c1.data(), C.v1.data());
    const double rho1 = dot(C.c1.data(), C.v1.data(), nc);
    const double a1 = dot(C.c1.data(), C.r.data(), nc);
    if (!(rho1 > 0.0)) fail("K-cycle: c1' A_c c1 <= 0");
#pragma omp parallel for schedule(static, 4096)
    for (int i = 0; i < nc; ++i) C.rt[i] = C.r[i] - (a1 / rho1) * C.v1[i];
    bh_kcycle(H, l + 1, C.rt.data(), C.c2.data());
    spmv(C.A, C.c2.data(), C.v2.data());
    const double gam = dot(C.c2.data(), C.v1.data(), nc);
    const double bet = dot(C.c2.data(), C.v2.data(), nc);
    const double a2 = dot(C.c2.data(), C.rt.data(), nc);
    const double rho2 = bet - gam * gam / rho1;
    if (rho2 > 0.0) {
      const double f1 = a1 / rho1 - gam * a2 / (rho1 * rho2), f2 = a2 / rho2;
#pragma omp parallel for schedule(static, 4096)
      for (int i = 0; i < nc; ++i) C.x[i] = f1 * C.c1[i] + f2 * C.c2[i];
    } else {  // c2 adds nothing A_c-independent of c1: one iteration
#pragma omp parallel for schedule(static, 4096)
      for (int i = 0; i < nc; ++i) C.x[i] = (a1 / rho1) * C.c1[i];
    }
  }
#pragma omp parallel for schedule(static, 4096)
  for (int i = 0; i < n; ++i) x[i] += L.P.p[i] * C.x[L.P.agg[i]];
  gs_sweep(L.A, L.d, L.C, r, x, false);
}

// ------------------------------------------------------ multi-vector levels

struct MvLevel {
  Csr A;
  GsOrder O;
  // transfer to the next level
  int nagg = 0;
  std::vector<int> aptr, arows, coff, uoff;
  std::vector<double> U, drop2;
  std::vector<double> W;  // n x nvec, row-major
};

// One-sided Jacobi SVD (Hestenes) of the na x m row-major matrix G (in place).
// On return the columns of G are U * Sigma (unsorted); sig holds the column norms.
void hestenes(std::vector<double>& G, int na, int m, std::vector<double>& sig) {
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        double alpha = 0, beta = 0, gamma = 0;
        for (int i = 0; i < na; ++i) {
          const double gp = G[(size_t)i * m + p], gq = G[(size_t)i * m + q];
          alpha += gp * gp;
          beta += gq * gq;
          gamma += gp * gq;
        }
        if (gamma == 0.0 || std::fabs(gamma) <= 1e-15 * std::sqrt(alpha * beta)) continue;
        rotated = true;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < na; ++i) {
          const double gp = G[(size_t)i * m + p], gq = G[(size_t)i * m + q];
          G[(size_t)i * m + p] = c * gp - s * gq;
          G[(size_t)i * m + q] = s * gp + c * gq;
        }
      }
    if (!rotated) break;
  }
  sig.assign(m, 0.0);
  for (int j = 0; j < m; ++j) {
    double s = 0;
    for (int i = 0; i < na; ++i) s += G[(size_t)i * m + j] * G[(size_t)i * m + j];
    sig[j] = std::sqrt(s);
  }
}

// Local basis of the smooth vectors on one aggregate (Section 4, eq. 4.3):
// left singular vectors with sigma > tol_a, at least one, at most na; columns
// re-orthonormalised (two Gram-Schmidt passes) and sign-fixed so that the
// entry of largest magnitude is positive.  Returns k; U is na x k row-major.
int aggregate_basis(const double* Pa, int na, int m, double tol_a, std::vector<double>& U,
                    double& drop2) {
  std::vector<double> G(Pa, Pa + (size_t)na * m), sig;
  hestenes(G, na, m, sig);
  std::vector<int> ord(m);
  for (int j = 0; j < m; ++j) ord[j] = j;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return sig[a] > sig[b]; });
  int k = 0;
  while (k < m && k < na && sig[ord[k]] > tol_a) ++k;
  if (k == 0) k = 1;
  if (!(sig[ord[0]] > 0.0)) fail("aggregate with all smooth vectors zero");
  drop2 = 0.0;
  for (int j = k; j < m; ++j) drop2 += sig[ord[j]] * sig[ord[j]];
  U.assign((size_t)na * k, 0.0);
  for (int l = 0; l < k; ++l) {
    const int j = ord[l];
    for (int i = 0; i < na; ++i) U[(size_t)i * k + l] = G[(size_t)i * m + j] / sig[j];
  }
  for (int pass = 0; pass < 2; ++pass)
    for (int l = 0; l < k; ++l) {
      for (int q = 0; q < l; ++q) {
        double h = 0;
        for (int i = 0; i < na; ++i) h += U[(size_t)i * k + q] * U[(size_t)i * k + l];
        for (int i = 0; i < na; ++i) U[(size_t)i * k + l] -= h * U[(size_t)i * k + q];
      }
      double s = 0;
      for (int i = 0; i < na; ++i) s += U[(size_t)i * k + l] * U[(size_t)i * k + l];
      s = std::sqrt(s);
      if (!(s > 0.0)) fail("rank loss while orthonormalising an aggregate basis");
      for (int i = 0; i < na; ++i) U[(size_t)i * k + l] /= s;
    }
  for (int l = 0; l < k; ++l) {
    int imax = 0;
    for (int i = 1; i < na; ++i)
      if (std::fabs(U[(size_t)i * k + l]) > std::fabs(U[(size_t)imax * k + l])) imax = i;
    if (U[(size_t)imax * k + l] < 0.0)
      for (int i = 0; i < na; ++i) U[(size_t)i * k + l] = -U[(size_t)i * k + l];
  }
  return k;
}

// Galerkin product P^T A P with block-diagonal P = blockdiag(U_a).
Csr galerkin_block(const Csr& A, const MvLevel& M, int nc, const std::vector<int>& agg_of,
                   const std::vector<int>& loc) {
  std::vector<std::vector<int>> cols(nc);
  std::vector<std::vector<double>> vals(nc);
#pragma omp parallel
  {
    std::vector<int> mark(M.nagg, -1);
    std::vector<int> nb, off;
    std::vector<double> T;
#pragma omp for schedule(dynamic, 64)
    for (int a = 0; a < M.nagg; ++a) {
      const int ka = M.coff[a + 1] - M.coff[a];
      nb.clear();
      for (int q = M.aptr[a]; q < M.aptr[a + 1]; ++q) {
        const int i = M.arows[q];
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
          const int b = agg_of[A.ci[k]];
          if (mark[b] < 0) {
            mark[b] = 0;
            nb.push_back(b);
          }
        }
      }
      std::sort(nb.begin(), nb.end());
      off.assign(nb.size() + 1, 0);
      for (size_t t = 0; t < nb.size(); ++t) {
        mark[nb[t]] = (int)t;
        off[t + 1] = off[t] + (M.coff[nb[t] + 1] - M.coff[nb[t]]);
      }
      const int K = off[nb.size()];
      T.assign((size_t)ka * K, 0.0);
      const double* Ua = M.U.data() + M.uoff[a];
      for (int q = M.aptr[a]; q < M.aptr[a + 1]; ++q) {
        const int i = M.arows[q];
        const int li = q - M.aptr[a];
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
          const int j = A.ci[k];
          const int b = agg_of[j];
          const int t = mark[b];
          const int kb = M.coff[b + 1] - M.coff[b];
          const double* Ub = M.U.data() + M.uoff[b] + (size_t)loc[j] * kb;
          for (int l = 0; l < ka; ++l) {
            const double f = Ua[(size_t)li * ka + l] * A.v[k];
            double* Trow = T.data() + (size_t)l * K + off[t];
            for (int mm = 0; mm < kb; ++mm) Trow[mm] += f * Ub[mm];
          }
        }
      }
      for (int l = 0; l < ka; ++l) {
        const int I = M.coff[a] + l;
        cols[I].resize(K);
        vals[I].resize(K);
        for (size_t t = 0; t < nb.size(); ++t) {
          const int kb = M.coff[nb[t] + 1] - M.coff[nb[t]];
          for (int mm = 0; mm < kb; ++mm) {
            cols[I][off[t] + mm] = M.coff[nb[t]] + mm;
            vals[I][off[t] + mm] = T[(size_t)l * K + off[t] + mm];
          }
        }
      }
      for (int b : nb) mark[b] = -1;
    }
  }
  Csr Ac = assemble(nc, cols, vals);
  symmetrize(Ac);
  return Ac;
}

// ------------------------------------------------------------- file output

struct Chunk {
  std::string name;
  uint32_t dtype;  // 1 int32, 2 float64, 3 int64
  const void* data;
  uint64_t count;
};

void write_file(const char* path, const std::vector<Chunk>& chunks) {
  FILE* f = std::fopen(path, "wb");
  if (!f) fail(std::string("cannot open output file ") + path);
  const char magic[8] = {'M', 'V', 'A', 'M', 'G', 'H', '0', '1'};
  const uint32_t version = 1, nch = (uint32_t)chunks.size();
  bool ok = std::fwrite(magic, 1, 8, f) == 8;
  ok = ok && std::fwrite(&version, 4, 1, f) == 1 && std::fwrite(&nch, 4, 1, f) == 1;
  for (const Chunk& c : chunks) {
    char name[48] = {0};
    std::strncpy(name, c.name.c_str(), 47);
    const uint32_t res = 0;
    const size_t es = (c.dtype == 1) ? 4 : 8;
    ok = ok && std::fwrite(name, 1, 48, f) == 48;
    ok = ok && std::fwrite(&c.dtype, 4, 1, f) == 1 && std::fwrite(&res, 4, 1, f) == 1;
    ok = ok && std::fwrite(&c.count, 8, 1, f) == 1;
    if (c.count) ok = ok && std::fwrite(c.data, es, c.count, f) == c.count;
    const size_t pad = (8 - (es * c.count) % 8) % 8;
    const char zeros[8] = {0};
    if (pad) ok = ok && std::fwrite(zeros, 1, pad, f) == pad;
  }
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) fail(std::string("write error on ") + path);
}

// Writes the bootstrap operator B_r (one hierarchy of Algorithm 1) in the
// same file format as the multiple-vector hierarchy: per level the matrix,
// its Gauss-Seidel order (the greedy colouring: every row its own group, the
// colours as stages, which is the order gs_sweep relaxes in), and the
// transfer as aggregates with one column each -- the composite pairwise
// prolongator's values on the aggregate's members, of unit norm per
// aggregate.  The meta record marks the file as stage `stage` of a bootstrap.
void write_boot_hierarchy(const BHier& H, const char* path, int stage) {
  const int L = (int)H.lv.size() - 1;
  std::vector<Chunk> ch;
  std::vector<int64_t> meta = {1, L + 1, 1, H.lv[0].A.n, (int64_t)H.lv[0].A.nnz(), 0, (int64_t)stage};
  std::vector<double> prmv = {0.0, 0.0, 0.0, 1.0, 0.0, 0.0};
  std::vector<double> st = {0.0, 0.0};
  std::vector<double> none;
  ch.push_back({"meta", 3, meta.data(), meta.size()});
  ch.push_back({"params", 2, prmv.data(), prmv.size()});
  ch.push_back({"stats", 2, st.data(), st.size()});
  ch.push_back({"rho", 2, none.data(), 0});
  struct Tr {
    std::vector<int> gptr, aptr, arows, coff, uoff;
    std::vector<double> U, drop2;
  };
  std::vector<Tr> tr(L);
  auto nm = [&](const char* f, int l) {
    char b[64];
    std::snprintf(b, sizeof b, f, l);
    return std::string(b);
  };
  for (int l = 0; l < L; ++l) {
    const BLevel& B = H.lv[l];
    Tr& T = tr[l];
    const int n = B.A.n, nc = B.P.nc;
    T.gptr.resize(n + 1);
    for (int i = 0; i <= n; ++i) T.gptr[i] = i;
    T.aptr.assign(nc + 1, 0);
    for (int i = 0; i < n; ++i) T.aptr[B.P.agg[i] + 1]++;
    for (int a = 0; a < nc; ++a) T.aptr[a + 1] += T.aptr[a];
    T.arows.resize(n);
    T.U.resize(n);
    std::vector<int> pos(T.aptr.begin(), T.aptr.end() - 1);
    for (int i = 0; i < n; ++i) {
      const int q = pos[B.P.agg[i]]++;
      T.arows[q] = i;
      T.U[q] = B.P.p[i];
    }
    T.coff.resize(nc + 1);
    for (int a = 0; a <= nc; ++a) T.coff[a] = a;
    T.uoff = T.aptr;
    T.drop2.assign(nc, 0.0);
  }
  for (int l = 0; l <= L; ++l) {
    const Csr& A = H.lv[l].A;
    ch.push_back({nm("A%d.rowptr", l), 1, A.rp.data(), A.rp.size()});
    ch.push_back({nm("A%d.col", l), 1, A.ci.data(), A.ci.size()});
    ch.push_back({nm("A%d.val", l), 2, A.v.data(), A.v.size()});
    if (l == L) break;
    const Colouring& C = H.lv[l].C;
    const Tr& T = tr[l];
    ch.push_back({nm("A%d.order", l), 1, C.crows.data(), C.crows.size()});
    ch.push_back({nm("A%d.gptr", l), 1, T.gptr.data(), T.gptr.size()});
    ch.push_back({nm("A%d.sptr", l), 1, C.cptr.data(), C.cptr.size()});
    ch.push_back({nm("P%d.aptr", l), 1, T.aptr.data(), T.aptr.size()});
    ch.push_back({nm("P%d.arows", l), 1, T.arows.data(), T.arows.size()});
    ch.push_back({nm("P%d.coff", l), 1, T.coff.data(), T.coff.size()});
    ch.push_back({nm("P%d.uoff", l), 1, T.uoff.data(), T.uoff.size()});
    ch.push_back({nm("P%d.U", l), 2, T.U.data(), T.U.size()});
    ch.push_back({nm("P%d.drop2", l), 2, T.drop2.data(), T.drop2.size()});
  }
  write_file(path, ch);
}

}  // namespace

// ================================================================== C ABI

extern "C" {

struct mvsetup_params {
  int nvec_max, nu;
  double rho_des;
  int maxstage;
  double tol_svd;
  int compose, coarse_cap, boot_coarse_min, hier_stage, store_w, max_levels, nthreads;
  int fine_group;
  int boot_dense_max;  // 0: 4096
  int coarsest_max;    // 0: 8192
  int boot_kcycle;     // 1: K-cycles in the bootstrap's testing phase
};

const char* mvsetup_last_error(void) { return g_err.c_str(); }

// Builds the hierarchy of A (CSR, symmetric, positive diagonal) and writes it
// to `path`.  `x0` holds the random initial iterates of the bootstrap testing
// phase: (nvec_max - 1) vectors of length n, one after the other.  `stats`
// receives up to 64 doubles: [0] nlevels, [1] nvec, [2] opc, [3] cr,
// [4] nstages, [5..22] per-stage rho, [23] the stage whose hierarchy was
// composed (0 = first), [24..] per-level n, [44..] per-level nnz.
int mvsetup_build_boot(int n, const int* rowptr, const int* col, const double* val, const double* x0,
                       const mvsetup_params* prm_in, const char* path, double* stats, const char* boot_prefix);

int mvsetup_build(int n, const int* rowptr, const int* col, const double* val,
                  const double* x0, const mvsetup_params* prm_in, const char* path,
                  double* stats) {
  return mvsetup_build_boot(n, rowptr, col, val, x0, prm_in, path, stats, nullptr);
}

// As mvsetup_build; when boot_prefix is not null, also writes the hierarchy
// of every bootstrap stage r = 1, 2, ... (the operators B_r whose symmetrized
// multiplicative composite the testing phase applies) to
// "<boot_prefix>_b<r>.bin".
int mvsetup_build_boot(int n, const int* rowptr, const int* col, const double* val, const double* x0,
                       const mvsetup_params* prm_in, const char* path, double* stats, const char* boot_prefix) {
  try {
    if (!prm_in || n <= 0 || !rowptr || !col || !val || !path) fail("invalid argument");
    Params prm{prm_in->nvec_max, prm_in->nu,         prm_in->rho_des,
               prm_in->maxstage, prm_in->tol_svd,    prm_in->compose,
               prm_in->coarse_cap, prm_in->boot_coarse_min, prm_in->hier_stage,
               prm_in->store_w,  prm_in->max_levels, prm_in->fine_group,
               prm_in->boot_dense_max > 0 ? prm_in->boot_dense_max : 4096,
               prm_in->coarsest_max > 0 ? prm_in->coarsest_max : 8192,
               prm_in->boot_kcycle != 0};
    if (prm.nvec_max < 1 || prm.nu < 1 || prm.compose < 1 || prm.max_levels < 2 ||
        prm.fine_group < 1 || n % prm.fine_group != 0)
      fail("invalid setup parameters");
    if (prm_in->nthreads > 0) omp_set_num_threads(prm_in->nthreads);
    Csr A;
    A.n = n;
    A.rp.assign(rowptr, rowptr + n + 1);
    if (A.rp[0] != 0) fail("rowptr[0] must be 0");
    for (int i = 0; i < n; ++i)
      if (A.rp[i + 1] < A.rp[i]) fail("rowptr not monotone");
    A.ci.assign(col, col + A.rp[n]);
    A.v.assign(val, val + A.rp[n]);
    for (int i = 0; i < n; ++i)
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        if (A.ci[k] < 0 || A.ci[k] >= n) fail("column index out of range");
        if (k > A.rp[i] && A.ci[k] <= A.ci[k - 1]) fail("column indices must be strictly increasing");
        if (!std::isfinite(A.v[k])) fail("non-finite matrix value");
      }
    const std::vector<double> d0 = diag_of(A);
    // one line per bootstrap stage on stderr when MVSETUP_PROGRESS is set
    const bool progress = std::getenv("MVSETUP_PROGRESS") != nullptr;

    // ---- bootstrap (Algorithm 1)
    std::vector<std::vector<double>> W;
    W.emplace_back(n, 1.0);  // w_0 = 1 (Section 5)
    std::vector<BHier> hs;
    std::vector<double> rhos;
    std::vector<double> Ax(n), Bz(n);
    const int stages_max = std::min(prm.maxstage, prm.nvec_max - 1);
    for (int r = 1; r <= stages_max; ++r) {
      hs.push_back(build_bootstrap_hierarchy(A, W.back(), prm));
      std::vector<double> x(x0 + (size_t)(r - 1) * n, x0 + (size_t)r * n), xprev(n);
      auto apply_factor = [&](BHier& H) {  // x <- (I - B A) x
        spmv(A, x.data(), Ax.data());
        if (prm.boot_kcycle)
          bh_kcycle(H, 0, Ax.data(), Bz.data());
        else
          bh_vcycle(H, 0, Ax.data(), Bz.data());
#pragma omp parallel for schedule(static, 4096)
        for (int i = 0; i < n; ++i) x[i] -= Bz[i];
      };
      for (int j = 0; j < prm.nu; ++j) {
        xprev = x;
        for (int s = 0; s < r; ++s) apply_factor(hs[s]);
        for (int s = r - 1; s >= 0; --s) apply_factor(hs[s]);
      }
      spmv(A, x.data(), Ax.data());
      const double an = std::sqrt(std::max(0.0, dot(x.data(), Ax.data(), n)));
      spmv(A, xprev.data(), Ax.data());
      const double ap = std::sqrt(std::max(0.0, dot(xprev.data(), Ax.data(), n)));
      const double rho = (ap > 0.0) ? an / ap : 0.0;
      rhos.push_back(rho);
      if (progress)
        std::fprintf(stderr, "mvsetup: stage %d: %d bootstrap levels (coarsest %d rows%s), rho %.3f\n", r,
                     (int)hs.back().lv.size(), hs.back().ncoarse, hs.back().stalled ? ", stalled" : "", rho);
      if (!(an > 0.0)) break;  // the composite solver is exact: nothing left to learn
      for (int i = 0; i < n; ++i) x[i] /= an;
      W.push_back(std::move(x));
      if (rho < prm.rho_des) break;
      if (r < stages_max) {
        // only the hierarchy that will be composed must be kept whole
      }
    }
    const int nvec = (int)W.size();
    if (boot_prefix)
      for (size_t r = 0; r < hs.size(); ++r)
        write_boot_hierarchy(hs[r], (std::string(boot_prefix) + "_b" + std::to_string(r + 1) + ".bin").c_str(),
                             (int)r + 1);
    // ---- multiple-vector hierarchy (Section 4), from the levels of one
    // bootstrap hierarchy H
    auto compose_levels = [&](const BHier& H) {
    const int D = (int)H.lv.size() - 1;  // index of the bootstrap coarsest level
    std::vector<MvLevel> mv(1);
    mv[0].A = A;
    mv[0].W.assign((size_t)n * nvec, 0.0);
    for (int i = 0; i < n; ++i)
      for (int r = 0; r < nvec; ++r) mv[0].W[(size_t)i * nvec + r] = W[r][i];
    std::vector<int> bnode(n);
    for (int i = 0; i < n; ++i) bnode[i] = i;
    int t = 0;
    for (int l = 0;; ++l) {
      MvLevel& M = mv[l];
      const int nl = M.A.n;
      if ((l > 0 && nl <= prm.coarse_cap) || t >= D) break;
      const int tn = std::min(t + prm.compose, D);
      // composite aggregate map of bootstrap nodes at level t -> level tn
      const int nb_t = H.lv[t].A.n;
      std::vector<int> cmap(nb_t);
      for (int x = 0; x < nb_t; ++x) {
        int y = x;
        for (int s = t; s < tn; ++s) y = H.lv[s].P.agg[y];
        cmap[x] = y;
      }
      M.nagg = H.lv[tn].A.n;
      std::vector<int> agg_of(nl);
      for (int q = 0; q < nl; ++q) agg_of[q] = cmap[bnode[q]];
      members(agg_of, M.nagg, M.aptr, M.arows);
      std::vector<int> loc(nl);
      for (int a = 0; a < M.nagg; ++a) {
        if (M.aptr[a + 1] == M.aptr[a]) fail("empty aggregate");
        for (int q = M.aptr[a]; q < M.aptr[a + 1]; ++q) loc[M.arows[q]] = q - M.aptr[a];
      }
      std::vector<std::vector<double>> Ublk(M.nagg);
      std::vector<int> kk(M.nagg);
      M.drop2.assign(M.nagg, 0.0);
      bool err = false;
      std::string emsg;
#pragma omp parallel
      {
        std::vector<double> Pa;
#pragma omp for schedule(dynamic, 64)
        for (int a = 0; a < M.nagg; ++a) {
          const int na = M.aptr[a + 1] - M.aptr[a];
          Pa.resize((size_t)na * nvec);
          for (int li = 0; li < na; ++li) {
            const int q = M.arows[M.aptr[a] + li];
            for (int r = 0; r < nvec; ++r) Pa[(size_t)li * nvec + r] = M.W[(size_t)q * nvec + r];
          }
          const double tol_a = prm.tol_svd * (double)na / (double)nl;
          try {
            kk[a] = aggregate_basis(Pa.data(), na, nvec, tol_a, Ublk[a], M.drop2[a]);
          } catch (const Fail& f) {
#pragma omp critical
            {
              err = true;
              emsg = f.msg;
            }
          }
        }
      }
      if (err) fail(emsg);
      M.coff.assign(M.nagg + 1, 0);
      M.uoff.assign(M.nagg + 1, 0);
      for (int a = 0; a < M.nagg; ++a) {
        M.coff[a + 1] = M.coff[a] + kk[a];
        M.uoff[a + 1] = M.uoff[a] + (int)Ublk[a].size();
      }
      M.U.resize(M.uoff[M.nagg]);
      for (int a = 0; a < M.nagg; ++a) std::copy(Ublk[a].begin(), Ublk[a].end(), M.U.begin() + M.uoff[a]);
      const int nc = M.coff[M.nagg];
      MvLevel next;
      next.A = galerkin_block(M.A, M, nc, agg_of, loc);
      next.W.assign((size_t)nc * nvec, 0.0);
      for (int a = 0; a < M.nagg; ++a) {
        const int ka = kk[a];
        for (int li = 0; li < M.aptr[a + 1] - M.aptr[a]; ++li) {
          const int q = M.arows[M.aptr[a] + li];
          for (int ll = 0; ll < ka; ++ll) {
            const double u = M.U[M.uoff[a] + (size_t)li * ka + ll];
            for (int r = 0; r < nvec; ++r)
              next.W[(size_t)(M.coff[a] + ll) * nvec + r] += u * M.W[(size_t)q * nvec + r];
          }
        }
      }
      {
        std::vector<int> gstart;
        if (l == 0) {
          for (int i = 0; i <= nl; i += prm.fine_group) gstart.push_back(i);
        } else {
          gstart = mv[l - 1].coff;
        }
        M.O = group_order(M.A, gstart);
      }
      std::vector<int> nbnode(nc);
      for (int a = 0; a < M.nagg; ++a)
        for (int ll = M.coff[a]; ll < M.coff[a + 1]; ++ll) nbnode[ll] = a;
      bnode.swap(nbnode);
      t = tn;
      mv.push_back(std::move(next));
    }
    return mv;
    };
    // The paper composes the first hierarchy; by default the last one is
    // composed, and if its levels cannot get down to a coarsest level of at
    // most coarsest_max rows (its own coarsening stalled above that), the
    // latest earlier one whose levels can.
    int hsel = (prm.hier_stage < 0) ? (int)hs.size() - 1 : std::min(prm.hier_stage, (int)hs.size() - 1);
    std::vector<MvLevel> mv;
    for (;; --hsel) {
      if (progress) std::fprintf(stderr, "mvsetup: composing the levels of stage %d\n", hsel + 1);
      mv = compose_levels(hs[hsel]);
      if (mv.back().A.n <= prm.coarsest_max || prm.hier_stage >= 0 || hsel == 0) break;
    }
    W.clear();
    A = Csr();
    const int L = (int)mv.size() - 1;
    if (mv[L].A.n > prm.coarsest_max)
      fail("coarsest level larger than " + std::to_string(prm.coarsest_max) +
           " rows; raise compose or lower coarse_cap");

    // ---- statistics
    double nnz_tot = 0, cr = 0;
    for (int l = 0; l <= L; ++l) nnz_tot += (double)mv[l].A.nnz();
    for (int l = 1; l <= L; ++l) cr += (double)mv[l - 1].A.n / (double)mv[l].A.n;
    if (stats) {
      for (int q = 0; q < 64; ++q) stats[q] = 0;
      stats[0] = L + 1;
      stats[1] = nvec;
      stats[2] = nnz_tot / (double)mv[0].A.nnz();
      stats[3] = (L > 0) ? cr / L : 0.0;
      stats[4] = (double)rhos.size();
      for (size_t s = 0; s < rhos.size() && s < 18; ++s) stats[5 + s] = rhos[s];
      stats[23] = hsel;
      for (int l = 0; l <= L && l < 20; ++l) {
        stats[24 + l] = mv[l].A.n;
        stats[44 + l] = (double)mv[l].A.nnz();
      }
    }

    // ---- write
    std::vector<Chunk> ch;
    std::vector<int64_t> meta = {1, L + 1, nvec, n, (int64_t)mv[0].A.nnz(), (int64_t)rhos.size(),
                                 (int64_t)hsel};
    std::vector<double> prmv = {prm.tol_svd, (double)prm.nu, prm.rho_des, (double)prm.compose,
                                (double)prm.coarse_cap, (double)prm.boot_coarse_min};
    std::vector<double> st = {stats ? stats[2] : 0.0, stats ? stats[3] : 0.0};
    ch.push_back({"meta", 3, meta.data(), meta.size()});
    ch.push_back({"params", 2, prmv.data(), prmv.size()});
    ch.push_back({"stats", 2, st.data(), st.size()});
    ch.push_back({"rho", 2, rhos.data(), rhos.size()});
    std::vector<std::string> names;
    names.reserve(16 * (L + 1));
    auto nm = [&](const char* f, int l) {
      char b[64];
      std::snprintf(b, sizeof b, f, l);
      return std::string(b);
    };
    for (int l = 0; l <= L; ++l) {
      const MvLevel& M = mv[l];
      ch.push_back({nm("A%d.rowptr", l), 1, M.A.rp.data(), M.A.rp.size()});
      ch.push_back({nm("A%d.col", l), 1, M.A.ci.data(), M.A.ci.size()});
      ch.push_back({nm("A%d.val", l), 2, M.A.v.data(), M.A.v.size()});
      if (prm.store_w) ch.push_back({nm("W%d", l), 2, M.W.data(), M.W.size()});
      if (l == L) break;
      ch.push_back({nm("A%d.order", l), 1, M.O.order.data(), M.O.order.size()});
      ch.push_back({nm("A%d.gptr", l), 1, M.O.gptr.data(), M.O.gptr.size()});
      ch.push_back({nm("A%d.sptr", l), 1, M.O.sptr.data(), M.O.sptr.size()});
      ch.push_back({nm("P%d.aptr", l), 1, M.aptr.data(), M.aptr.size()});
      ch.push_back({nm("P%d.arows", l), 1, M.arows.data(), M.arows.size()});
      ch.push_back({nm("P%d.coff", l), 1, M.coff.data(), M.coff.size()});
      ch.push_back({nm("P%d.uoff", l), 1, M.uoff.data(), M.uoff.size()});
      ch.push_back({nm("P%d.U", l), 2, M.U.data(), M.U.size()});
      ch.push_back({nm("P%d.drop2", l), 2, M.drop2.data(), M.drop2.size()});
    }
    write_file(path, ch);
    return 0;
  } catch (const Fail& f) {
    g_err = f.msg;
    return -1;
  } catch (const std::exception& e) {
    g_err = e.what();
    return -1;
  }
}

// One pairwise aggregation step (Section 3), exposed for tests: agg (n),
// p (n), returns the number of coarse nodes or -1.
int mvsetup_pairwise(int n, const int* rowptr, const int* col, const double* val,
                     const double* w, int* agg, double* p) {
  try {
    Csr A;
    A.n = n;
    A.rp.assign(rowptr, rowptr + n + 1);
    A.ci.assign(col, col + A.rp[n]);
    A.v.assign(val, val + A.rp[n]);
    std::vector<double> d = diag_of(A);
    std::vector<double> wv(w, w + n);
    PcMap P = pairwise(A, d, wv);
    std::copy(P.agg.begin(), P.agg.end(), agg);
    std::copy(P.p.begin(), P.p.end(), p);
    return P.nc;
  } catch (const Fail& f) {
    g_err = f.msg;
    return -1;
  }
}

// Solves A x = b with the sparse Cholesky factor of a stalled coarsest level
// (A symmetric positive definite, CSR with sorted columns).  Returns the
// number of off-diagonal entries of L, or -1 (error text in
// mvsetup_last_error).
int64_t mvsetup_sparse_solve(int n, const int* rowptr, const int* col, const double* val, const double* b,
                             double* x) {
  try {
    if (n <= 0 || !rowptr || !col || !val || !b || !x) fail("invalid argument");
    Csr A;
    A.n = n;
    A.rp.assign(rowptr, rowptr + n + 1);
    A.ci.assign(col, col + A.rp[n]);
    A.v.assign(val, val + A.rp[n]);
    const SparseChol F = sparse_cholesky(A);
    sparse_cholesky_solve(F, b, x);
    return F.lp[n];
  } catch (const Fail& f) {
    g_err = f.msg;
    return -1;
  }
}

// Matching edge weights c_ij for every stored entry (diagonal entries get -1).
int mvsetup_edge_weights(int n, const int* rowptr, const int* col, const double* val,
                         const double* w, double* c) {
  try {
    Csr A;
    A.n = n;
    A.rp.assign(rowptr, rowptr + n + 1);
    A.ci.assign(col, col + A.rp[n]);
    A.v.assign(val, val + A.rp[n]);
    std::vector<double> d = diag_of(A);
    for (int i = 0; i < n; ++i)
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int j = A.ci[k];
        if (j == i) {
          c[k] = -1.0;
          continue;
        }
        const int lo = std::min(i, j), hi = std::max(i, j);
        c[k] = edge_weight(A.v[k], d[lo], d[hi], w[lo], w[hi]);
      }
    return 0;
  } catch (const Fail& f) {
    g_err = f.msg;
    return -1;
  }
}

// Per-aggregate basis (Section 4, eq. 4.3) exposed for tests: Pa is na x m
// row-major; U receives na x k (row-major, capacity na*m); returns k or -1.
int mvsetup_aggregate_basis(const double* Pa, int na, int m, double tol_a, double* U,
                            double* drop2) {
  try {
    std::vector<double> Uv;
    double d2 = 0;
    const int k = aggregate_basis(Pa, na, m, tol_a, Uv, d2);
    std::copy(Uv.begin(), Uv.end(), U);
    *drop2 = d2;
    return k;
  } catch (const Fail& f) {
    g_err = f.msg;
    return -1;
  }
}

}  // extern "C"
