// Composite AMG over several hierarchies B_1..B_r of the same fine matrix:
// the bootstrap's own solver (eq. 1.1, Algorithm 1, Section 5 item (i)).
// Its error propagator is the symmetrized multiplicative product
//   I - B A = (I - B_1 A)..(I - B_r A)(I - B_r A)..(I - B_1 A),
// applied factor by factor, rightmost first.  Every hierarchy keeps its own
// smoother-order numbering of the fine rows, so the composite works on
// file-order vectors in the caller's work space and each factor gathers into
// and scatters out of its hierarchy's numbering.  Products with A use the
// first hierarchy's fine level.  Included inside mvamg_lib.hip's anonymous
// namespace.

// file-order vectors of the work space: t, z (apply) and r, p, q, y (CG), then
// the partial sums and the scalars of the reductions
constexpr int kCompVecs = 6;
constexpr int kCompParts = 3 * 512;

size_t composite_work_bytes(int n) {
  const size_t v = ((size_t)n * sizeof(double) + 255) / 256 * 256;
  return kCompVecs * v + (size_t)(kCompParts + 16) * sizeof(double);
}

struct CompWork {
  double *t, *z, *r, *p, *q, *y, *part, *scal;
};

CompWork comp_work(int n, void* work, size_t bytes) {
  if (!work) throw Error(MVAMG_ERR_ARG, "null work space");
  if (reinterpret_cast<uintptr_t>(work) % 256 != 0) throw Error(MVAMG_ERR_ARG, "work space must be 256-byte aligned");
  if (bytes < composite_work_bytes(n))
    throw Error(MVAMG_ERR_ARG, "work space of " + std::to_string(bytes) + " bytes is too small (needs " +
                                   std::to_string(composite_work_bytes(n)) + ")");
  const size_t v = ((size_t)n * sizeof(double) + 255) / 256 * 256;
  unsigned char* b = (unsigned char*)work;
  CompWork w;
  double** slots[kCompVecs] = {&w.t, &w.z, &w.r, &w.p, &w.q, &w.y};
  for (int k = 0; k < kCompVecs; ++k) *slots[k] = (double*)(b + k * v);
  w.part = (double*)(b + kCompVecs * v);
  w.scal = w.part + kCompParts;
  return w;
}

// The r handles: one fine matrix (same size, pattern and values, checked on
// the device against the first), single problems, the current device.
void check_composite(mvamg_hier* const* hs, int r, hipStream_t st) {
  if (!hs || r < 1) throw Error(MVAMG_ERR_ARG, "no hierarchies");
  for (int k = 0; k < r; ++k) {
    if (!hs[k]) throw Error(MVAMG_ERR_ARG, "null hierarchy");
    if (hs[k]->nprob > 0) throw Error(MVAMG_ERR_ARG, "batch handles cannot form a composite");
    check_device(hs[k]);
    if (hs[k]->n != hs[0]->n || hs[k]->nnz != hs[0]->nnz)
      throw Error(MVAMG_ERR_ARG, "the hierarchies are not built on the same fine matrix");
  }
  mvamg_hier* h0 = hs[0];
  k_fill<int><<<1, kBlock, 0, st>>>(2, 0, h0->cmpflag);
  for (int k = 1; k < r; ++k) {
    k_differs<int><<<grid_for(h0->n + 1), kBlock, 0, st>>>(h0->n + 1, hs[k]->frp, h0->frp, h0->cmpflag);
    k_differs<int><<<grid_for(h0->nnz), kBlock, 0, st>>>(h0->nnz, hs[k]->fci, h0->fci, h0->cmpflag);
    k_differs<double><<<grid_for(h0->nnz), kBlock, 0, st>>>(h0->nnz, hs[k]->fval, h0->fval, h0->cmpflag);
  }
  LAUNCHCHECK("check_composite");
  int flags[2] = {0, 0};
  HIPCHECK(hipMemcpyAsync(flags, h0->cmpflag, sizeof(flags), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  if (flags[0]) throw Error(MVAMG_ERR_ARG, "the hierarchies are not built on the same fine matrix");
}

// y = A x for file-order vectors, with the first hierarchy's fine level
void comp_spmv(mvamg_hier* h0, const double* x, double* y, hipStream_t st) {
  const int eg = grid_for(h0->n);
  k_gather<<<eg, kBlock, 0, st>>>(h0->n, h0->perm0, x, h0->p);
  resid<double, 2>(h0, 0, h0->lv[0], nullptr, h0->p, h0->q, M_NONE, st);
  k_scatter<<<eg, kBlock, 0, st>>>(h0->n, h0->perm0, h0->q, y);
  LAUNCHCHECK("comp_spmv");
}

// out (file order) += sign * B_k t (file order)
void comp_component(mvamg_hier* hk, const double* t, double* out, double sign, int cycle, int smoother,
                    hipStream_t st) {
  const int eg = grid_for(hk->n);
  k_gather<<<eg, kBlock, 0, st>>>(hk->n, hk->perm0, t, hk->r);
  apply_B(hk, hk->r, hk->z, 64, smoother, st, cycle);
  k_scatter_axpy<<<eg, kBlock, 0, st>>>(hk->n, hk->perm0, sign, hk->z, out);
  LAUNCHCHECK("comp_component");
}

// factor order of the symmetrized product: 1, 2, .., r, r, .., 2, 1 (0-based)
int comp_index(int r, int j) { return j < r ? j : 2 * r - 1 - j; }

// z = B res (file order): from z = 0, every factor k takes z += B_k (res - A z)
void comp_apply(mvamg_hier* const* hs, int r, int cycle, int smoother, const double* res, double* z,
                const CompWork& w, hipStream_t st) {
  const int n = hs[0]->n, eg = grid_elem(n);
  k_fill<double><<<eg, kBlock, 0, st>>>(n, 0.0, z);
  for (int j = 0; j < 2 * r; ++j) {
    comp_spmv(hs[0], z, w.t, st);
    k_axpby<<<eg, kBlock, 0, st>>>(n, 1.0, res, -1.0, w.t, w.t);
    comp_component(hs[comp_index(r, j)], w.t, z, 1.0, cycle, smoother, st);
  }
}

// x.y (and u.v) summed on the device, returned on the host
void comp_dots(int n, const double* x, const double* y, const double* u, const double* v, double* out, int nv,
               const CompWork& w, hipStream_t st) {
  const int grid = std::min(grid_for(n), 512);
  if (nv == 1) {
    k_kdots<1><<<grid, kBlock, 0, st>>>(n, x, y, nullptr, nullptr, nullptr, nullptr, w.part);
    k_kfinish<1><<<1, kBlock, 0, st>>>(grid, w.part, w.scal);
  } else {
    k_kdots<2><<<grid, kBlock, 0, st>>>(n, x, y, u, v, nullptr, nullptr, w.part);
    k_kfinish<2><<<1, kBlock, 0, st>>>(grid, w.part, w.scal);
  }
  LAUNCHCHECK("comp_dots");
  HIPCHECK(hipMemcpyAsync(out, w.scal, nv * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
}

// The testing phase: x <- E x nu times, rho = ||x^nu||_A / ||x^{nu-1}||_A,
// x <- x^nu / ||x^nu||_A (x^nu when that norm is zero).
double comp_test(mvamg_hier* const* hs, int r, int cycle, int smoother, int nu, double* x, const CompWork& w,
                 hipStream_t st) {
  const int n = hs[0]->n, eg = grid_elem(n);
  for (int it = 0; it < nu; ++it) {
    k_copy<double><<<eg, kBlock, 0, st>>>(n, x, w.y);
    for (int j = 0; j < 2 * r; ++j) {
      comp_spmv(hs[0], x, w.t, st);
      comp_component(hs[comp_index(r, j)], w.t, x, -1.0, cycle, smoother, st);
    }
  }
  double an2 = 0.0, ap2 = 0.0;
  comp_spmv(hs[0], x, w.t, st);
  comp_dots(n, x, w.t, nullptr, nullptr, &an2, 1, w, st);
  comp_spmv(hs[0], w.y, w.t, st);
  comp_dots(n, w.y, w.t, nullptr, nullptr, &ap2, 1, w, st);
  const double an = std::sqrt(std::max(0.0, an2)), ap = std::sqrt(std::max(0.0, ap2));
  if (!std::isfinite(an) || !std::isfinite(ap)) throw Error(MVAMG_ERR_NONFINITE, "non-finite value in the testing phase");
  if (an > 0.0) {
    k_div<<<eg, kBlock, 0, st>>>(n, an, x);
    LAUNCHCHECK("comp_test");
  }
  HIPCHECK(hipStreamSynchronize(st));
  return ap > 0.0 ? an / ap : 0.0;
}

// CG preconditioned by the composite, flexible beta (K-cycle components are
// not linear): stopping rule, history and info as pcg.
mvamg_status comp_pcg(mvamg_hier* const* hs, int r, const double* b, double* x, const mvamg_solve_params* prm,
                      mvamg_info* info, const CompWork& w, hipStream_t st) {
  const int n = hs[0]->n, eg = grid_elem(n);
  mvamg_info inf{};
  comp_spmv(hs[0], x, w.q, st);
  k_axpby<<<eg, kBlock, 0, st>>>(n, 1.0, b, -1.0, w.q, w.r);
  double rr = 0.0;
  comp_dots(n, w.r, w.r, nullptr, nullptr, &rr, 1, w, st);
  const double r0 = std::sqrt(rr);
  if (!std::isfinite(r0)) throw Error(MVAMG_ERR_NONFINITE, "non-finite initial residual (check b and x0)");
  if (prm->history) prm->history[0] = 1.0;
  mvamg_status status = MVAMG_NOT_CONVERGED;
  double h_last = 1.0;
  if (r0 == 0.0) {
    status = MVAMG_OK;
    inf.converged = 1;
    h_last = 0.0;
  } else {
    comp_apply(hs, r, prm->cycle, prm->smoother, w.r, w.z, w, st);
    k_copy<double><<<eg, kBlock, 0, st>>>(n, w.z, w.p);
    double rho = 0.0;
    comp_dots(n, w.r, w.z, nullptr, nullptr, &rho, 1, w, st);
    int it = 0;
    while (it < prm->maxit) {
      comp_spmv(hs[0], w.p, w.q, st);
      double pq = 0.0;
      comp_dots(n, w.p, w.q, nullptr, nullptr, &pq, 1, w, st);
      if (!(pq > 0.0)) {
        inf.iterations = it;
        throw Error(MVAMG_ERR_BREAKDOWN, "CG breakdown: p^T A p <= 0 (matrix not s.p.d.)");
      }
      const double alpha = rho / pq;
      k_axpby<<<eg, kBlock, 0, st>>>(n, 1.0, x, alpha, w.p, x);
      k_axpby<<<eg, kBlock, 0, st>>>(n, 1.0, w.r, -alpha, w.q, w.r);
      comp_dots(n, w.r, w.r, nullptr, nullptr, &rr, 1, w, st);
      ++it;
      h_last = std::sqrt(rr) / r0;
      if (prm->history) prm->history[it] = h_last;
      if (!std::isfinite(h_last)) throw Error(MVAMG_ERR_NONFINITE, "non-finite residual during CG");
      if (h_last <= prm->rtol) {
        status = MVAMG_OK;
        break;
      }
      comp_apply(hs, r, prm->cycle, prm->smoother, w.r, w.z, w, st);
      double d[2] = {0.0, 0.0};  // z.q, r.z
      comp_dots(n, w.z, w.q, w.r, w.z, d, 2, w, st);
      const double beta = -alpha * d[0] / rho;
      rho = d[1];
      k_axpby<<<eg, kBlock, 0, st>>>(n, 1.0, w.z, beta, w.p, w.p);
      LAUNCHCHECK("comp_pcg");
    }
    inf.iterations = it;
    inf.converged = (status == MVAMG_OK);
  }
  inf.rel_res = h_last;
  comp_spmv(hs[0], x, w.q, st);
  k_axpby<<<eg, kBlock, 0, st>>>(n, 1.0, b, -1.0, w.q, w.q);
  comp_dots(n, w.q, w.q, nullptr, nullptr, &rr, 1, w, st);
  inf.rel_res_true = (r0 > 0.0) ? std::sqrt(rr) / r0 : 0.0;
  if (info) *info = inf;
  return status;
}
