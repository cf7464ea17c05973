/*
 * CPU oracle of the solve phase of the single-hierarchy multiple-vector
 * aggregation-based AMG (D'Ambra & Vassilevski).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may call it; the
 * product path never does.  It shares no code with the GPU library.
 *
 * Every loop follows the definition it cites, in that order, with no blocking
 * or fusion.  Build: gcc -O2 -ffp-contract=off (no FMA contraction).
 *
 *   orc_vcycle   z = B r, one V-cycle (Section 5: forward/backward
 *                Gauss-Seidel pre/post-smoothing on every level but the
 *                coarsest, exact coarsest solve; "standard V-cycle").
 *   orc_pcg      preconditioned conjugate gradient with B (Section 5), stop
 *                when ||r_k||_2 <= tol ||r_0||_2 or after maxit iterations.
 *   orc_vcycle32 / orc_pcg_mixed  the same cycle in binary32 arithmetic with a
 *                binary64 flexible PCG outside it (extension beyond the paper).
 *   orc_grad_coeffs  dL/da_ij = -lambda_i x_j on the sparsity pattern
 *                (adjoint of A x = b for symmetric A; extension).
 *   orc_kcycle / orc_pcg_kcycle  the K-cycle (nonlinear AMLI cycle) over the
 *                same hierarchy, and CG with it as preconditioner (Section 5:
 *                the bootstrap applies its AMG components as K-cycles with
 *                two inner flexible-CG iterations per level but the coarsest).
 *   orc_composite_apply / orc_composite_test / orc_pcg_composite  the
 *                bootstrap's composite AMG over several hierarchies B_1..B_r
 *                (eq. 1.1, Algorithm 1, Section 5 item (i): the symmetrized
 *                multiplicative product (I - B_1 A)..(I - B_r A)(I - B_r A)..
 *                (I - B_1 A)), its testing phase, and CG preconditioned by it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int n;
  const int* rowptr;
  const int* col;
  const double* val;
  /* Gauss-Seidel order of a non-coarsest level: the n rows in relaxation order */
  const int* order;
  /* block-diagonal prolongator to the next level (Section 4):
     aggregate a has members arows[aptr[a]..aptr[a+1]), coarse dofs
     coff[a]..coff[a+1]-1, and U_a (n_a x k_a, row-major) at U + uoff[a]. */
  int nagg;
  const int* aptr;
  const int* arows;
  const int* coff;
  const int* uoff;
  const double* U;
} orc_level;

enum { ORC_GS_COLOUR = 0, ORC_GS_LEX = 1, ORC_L1_JACOBI = 2 };

typedef struct {
  int nl;
  orc_level* lv; /* copy of the level descriptors (arrays borrowed) */
  int smoother;
  double* Lc; /* dense Cholesky factor of the coarsest matrix, row-major */
  int nL;
  /* binary32 copies for the mixed-precision cycle */
  float** val32;
  float** U32;
} orc_hier;

/* ------------------------------------------------------------ helpers */

static double dotp(const double* a, const double* b, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* y = A x */
static void csr_mv(int n, const int* rp, const int* ci, const double* v, const double* x, double* y) {
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) s += v[k] * x[ci[k]];
    y[i] = s;
  }
}

/* Dense Cholesky A = L L^T of the coarsest matrix (lower triangle). */
static int cholesky(double* M, int n) {
  for (int j = 0; j < n; ++j) {
    double s = M[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= M[(size_t)j * n + k] * M[(size_t)j * n + k];
    if (!(s > 0.0)) return -1;
    double ljj = sqrt(s);
    M[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = M[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= M[(size_t)i * n + k] * M[(size_t)j * n + k];
      M[(size_t)i * n + j] = t / ljj;
    }
  }
  return 0;
}

/* z = A_L^{-1} r: forward substitution with L, back substitution with L^T. */
static void chol_solve(const double* L, int n, const double* r, double* z) {
  double* y = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int i = 0; i < n; ++i) {
    double s = r[i];
    for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * y[k];
    y[i] = s / L[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * z[k];
    z[i] = s / L[(size_t)i * n + i];
  }
  free(y);
}

/* ------------------------------------------------------------ smoothers */

/* Gauss-Seidel update of row i: x_i <- (r_i - sum_{j != i} a_ij x_j) / a_ii */
static void gs_row(const orc_level* L, const double* val, const double* r, double* x, int i) {
  double s = r[i], d = 0.0;
  for (int k = L->rowptr[i]; k < L->rowptr[i + 1]; ++k) {
    int j = L->col[k];
    if (j == i)
      d = val[k];
    else
      s -= val[k] * x[j];
  }
  x[i] = s / d;
}

/* One Gauss-Seidel sweep in the order O: the level's stored order (rows grouped
   colour by colour) or lexicographic; backward = exact reverse of O. */
static void gs_sweep(const orc_hier* H, int l, const double* val, const double* r, double* x,
                     int forward) {
  const orc_level* L = &H->lv[l];
  if (H->smoother == ORC_GS_LEX) {
    if (forward)
      for (int i = 0; i < L->n; ++i) gs_row(L, val, r, x, i);
    else
      for (int i = L->n - 1; i >= 0; --i) gs_row(L, val, r, x, i);
    return;
  }
  const int n = L->n;
  if (forward)
    for (int q = 0; q < n; ++q) gs_row(L, val, r, x, L->order[q]);
  else
    for (int q = n - 1; q >= 0; --q) gs_row(L, val, r, x, L->order[q]);
}

/* l1-Jacobi (Baker, Falgout, Kolev, Yang 2011): x <- x + D_l1^{-1} (r - A x),
   d_i = sum_j |a_ij|. */
static void l1_jacobi(const orc_level* L, const double* val, const double* r, double* x) {
  double* t = (double*)malloc(sizeof(double) * (size_t)L->n);
  csr_mv(L->n, L->rowptr, L->col, val, x, t);
  for (int i = 0; i < L->n; ++i) {
    double d = 0.0;
    for (int k = L->rowptr[i]; k < L->rowptr[i + 1]; ++k) d += fabs(val[k]);
    t[i] = (r[i] - t[i]) / d;
  }
  for (int i = 0; i < L->n; ++i) x[i] += t[i];
  free(t);
}

/* ------------------------------------------------------------ transfers */

/* r_c = P^T s: r_c[coff_a + l] = sum_{i in a} U_a[i, l] s[i]  (P = blockdiag(U_a)) */
static void restrict_p(const orc_level* L, const double* s, double* rc) {
  for (int a = 0; a < L->nagg; ++a) {
    const int na = L->aptr[a + 1] - L->aptr[a], ka = L->coff[a + 1] - L->coff[a];
    const double* Ua = L->U + L->uoff[a];
    for (int l = 0; l < ka; ++l) {
      double acc = 0.0;
      for (int li = 0; li < na; ++li) acc += Ua[(size_t)li * ka + l] * s[L->arows[L->aptr[a] + li]];
      rc[L->coff[a] + l] = acc;
    }
  }
}

/* x += P x_c */
static void prolong_add(const orc_level* L, const double* xc, double* x) {
  for (int a = 0; a < L->nagg; ++a) {
    const int na = L->aptr[a + 1] - L->aptr[a], ka = L->coff[a + 1] - L->coff[a];
    const double* Ua = L->U + L->uoff[a];
    for (int li = 0; li < na; ++li) {
      double acc = 0.0;
      for (int l = 0; l < ka; ++l) acc += Ua[(size_t)li * ka + l] * xc[L->coff[a] + l];
      x[L->arows[L->aptr[a] + li]] += acc;
    }
  }
}

/* ------------------------------------------------------------ V-cycle */

/* x = B_l r.  val0 (may be NULL) replaces the stored values of level 0. */
static void vcycle(const orc_hier* H, int l, const double* val0, const double* r, double* x) {
  const orc_level* L = &H->lv[l];
  const int n = L->n;
  if (l == H->nl - 1) {
    chol_solve(H->Lc, n, r, x);
    return;
  }
  const double* val = (l == 0 && val0) ? val0 : L->val;
  const int nc = H->lv[l + 1].n;
  double* s = (double*)malloc(sizeof(double) * (size_t)n);
  double* rc = (double*)malloc(sizeof(double) * (size_t)nc);
  double* xc = (double*)malloc(sizeof(double) * (size_t)nc);
  for (int i = 0; i < n; ++i) x[i] = 0.0;
  /* pre-smoothing: one forward sweep */
  if (H->smoother == ORC_L1_JACOBI)
    l1_jacobi(L, val, r, x);
  else
    gs_sweep(H, l, val, r, x, 1);
  /* residual and restriction */
  csr_mv(n, L->rowptr, L->col, val, x, s);
  for (int i = 0; i < n; ++i) s[i] = r[i] - s[i];
  restrict_p(L, s, rc);
  /* coarse correction */
  vcycle(H, l + 1, val0, rc, xc);
  prolong_add(L, xc, x);
  /* post-smoothing: one backward sweep */
  if (H->smoother == ORC_L1_JACOBI)
    l1_jacobi(L, val, r, x);
  else
    gs_sweep(H, l, val, r, x, 0);
  free(s);
  free(rc);
  free(xc);
}

/* ------------------------------------------------------------ K-cycle */

static void kcycle(const orc_hier* H, int l, const double* val0, const double* r, double* x);

/* y ~ A_m^{-1} g by two iterations of flexible CG from y = 0, both
   preconditioned by the K-cycle of level m (Notay & Vassilevski 2008;
   Section 5 takes two inner iterations).  The first direction is c1 = K g;
   the second, c2 = K r2 with r2 = g - alpha1 A c1, is made A-orthogonal to
   c1, so y is the A-orthogonal projection of A_m^{-1} g on span{c1, c2}. */
static void kc_fcg2(const orc_hier* H, int m, const double* g, double* y) {
  const orc_level* L = &H->lv[m];
  const int n = L->n;
  double* c1 = (double*)calloc((size_t)n, sizeof(double));
  double* v1 = (double*)calloc((size_t)n, sizeof(double));
  double* r2 = (double*)calloc((size_t)n, sizeof(double));
  double* c2 = (double*)calloc((size_t)n, sizeof(double));
  double* v2 = (double*)calloc((size_t)n, sizeof(double));
  /* first iteration: y1 = alpha1 c1 */
  kcycle(H, m, NULL, g, c1);
  csr_mv(n, L->rowptr, L->col, L->val, c1, v1);
  const double rho1 = dotp(c1, v1, n);
  const double alpha1 = dotp(c1, g, n) / rho1;
  for (int i = 0; i < n; ++i) r2[i] = g[i] - alpha1 * v1[i];
  /* second iteration: direction p2 = c2 - (gamma / rho1) c1 */
  kcycle(H, m, NULL, r2, c2);
  csr_mv(n, L->rowptr, L->col, L->val, c2, v2);
  const double gamma = dotp(c2, v1, n);
  const double beta = dotp(c2, v2, n) - gamma * gamma / rho1; /* p2^T A p2 */
  const double alpha2 = dotp(c2, r2, n) / beta;
  /* y = alpha1 c1 + alpha2 p2 */
  const double t1 = alpha1 - alpha2 * gamma / rho1;
  for (int i = 0; i < n; ++i) y[i] = t1 * c1[i] + alpha2 * c2[i];
  free(c1);
  free(v1);
  free(r2);
  free(c2);
  free(v2);
}

/* x = K_l r: the V-cycle's smoothing and transfers, with the coarse
   correction on a level that is not the coarsest taken from kc_fcg2. */
static void kcycle(const orc_hier* H, int l, const double* val0, const double* r, double* x) {
  const orc_level* L = &H->lv[l];
  const int n = L->n;
  if (l == H->nl - 1) {
    chol_solve(H->Lc, n, r, x);
    return;
  }
  const double* val = (l == 0 && val0) ? val0 : L->val;
  const int nc = H->lv[l + 1].n;
  double* s = (double*)malloc(sizeof(double) * (size_t)n);
  double* rc = (double*)malloc(sizeof(double) * (size_t)nc);
  double* xc = (double*)malloc(sizeof(double) * (size_t)nc);
  for (int i = 0; i < n; ++i) x[i] = 0.0;
  if (H->smoother == ORC_L1_JACOBI)
    l1_jacobi(L, val, r, x);
  else
    gs_sweep(H, l, val, r, x, 1);
  csr_mv(n, L->rowptr, L->col, val, x, s);
  for (int i = 0; i < n; ++i) s[i] = r[i] - s[i];
  restrict_p(L, s, rc);
  if (l + 1 == H->nl - 1)
    chol_solve(H->Lc, nc, rc, xc);
  else
    kc_fcg2(H, l + 1, rc, xc);
  prolong_add(L, xc, x);
  if (H->smoother == ORC_L1_JACOBI)
    l1_jacobi(L, val, r, x);
  else
    gs_sweep(H, l, val, r, x, 0);
  free(s);
  free(rc);
  free(xc);
}

/* ------------------------------------------------------ binary32 cycle */

static void gs_row32(const orc_level* L, const float* val, const float* r, float* x, int i) {
  float s = r[i], d = 0.0f;
  for (int k = L->rowptr[i]; k < L->rowptr[i + 1]; ++k) {
    int j = L->col[k];
    if (j == i)
      d = val[k];
    else
      s -= val[k] * x[j];
  }
  x[i] = s / d;
}

static void gs_sweep32(const orc_hier* H, int l, const float* val, const float* r, float* x,
                       int forward) {
  const orc_level* L = &H->lv[l];
  if (H->smoother == ORC_GS_LEX) {
    if (forward)
      for (int i = 0; i < L->n; ++i) gs_row32(L, val, r, x, i);
    else
      for (int i = L->n - 1; i >= 0; --i) gs_row32(L, val, r, x, i);
    return;
  }
  const int n = L->n;
  if (forward)
    for (int q = 0; q < n; ++q) gs_row32(L, val, r, x, L->order[q]);
  else
    for (int q = n - 1; q >= 0; --q) gs_row32(L, val, r, x, L->order[q]);
}

static void l1_jacobi32(const orc_level* L, const float* val, const float* r, float* x) {
  float* t = (float*)malloc(sizeof(float) * (size_t)L->n);
  for (int i = 0; i < L->n; ++i) {
    float s = 0.0f, d = 0.0f;
    for (int k = L->rowptr[i]; k < L->rowptr[i + 1]; ++k) {
      s += val[k] * x[L->col[k]];
      d += fabsf(val[k]);
    }
    t[i] = (r[i] - s) / d;
  }
  for (int i = 0; i < L->n; ++i) x[i] += t[i];
  free(t);
}

static void vcycle32(const orc_hier* H, int l, const float* val0, const float* r, float* x) {
  const orc_level* L = &H->lv[l];
  const int n = L->n;
  if (l == H->nl - 1) {
    /* coarsest solve stays binary64 */
    double* rd = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double* xd = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int i = 0; i < n; ++i) rd[i] = (double)r[i];
    chol_solve(H->Lc, n, rd, xd);
    for (int i = 0; i < n; ++i) x[i] = (float)xd[i];
    free(rd);
    free(xd);
    return;
  }
  const float* val = (l == 0 && val0) ? val0 : H->val32[l];
  const float* U = H->U32[l];
  const int nc = H->lv[l + 1].n;
  float* s = (float*)malloc(sizeof(float) * (size_t)n);
  float* rc = (float*)malloc(sizeof(float) * (size_t)nc);
  float* xc = (float*)malloc(sizeof(float) * (size_t)nc);
  for (int i = 0; i < n; ++i) x[i] = 0.0f;
  if (H->smoother == ORC_L1_JACOBI)
    l1_jacobi32(L, val, r, x);
  else
    gs_sweep32(H, l, val, r, x, 1);
  for (int i = 0; i < n; ++i) {
    float t = 0.0f;
    for (int k = L->rowptr[i]; k < L->rowptr[i + 1]; ++k) t += val[k] * x[L->col[k]];
    s[i] = r[i] - t;
  }
  for (int a = 0; a < L->nagg; ++a) {
    const int na = L->aptr[a + 1] - L->aptr[a], ka = L->coff[a + 1] - L->coff[a];
    const float* Ua = U + L->uoff[a];
    for (int q = 0; q < ka; ++q) {
      float acc = 0.0f;
      for (int li = 0; li < na; ++li) acc += Ua[(size_t)li * ka + q] * s[L->arows[L->aptr[a] + li]];
      rc[L->coff[a] + q] = acc;
    }
  }
  vcycle32(H, l + 1, val0, rc, xc);
  for (int a = 0; a < L->nagg; ++a) {
    const int na = L->aptr[a + 1] - L->aptr[a], ka = L->coff[a + 1] - L->coff[a];
    const float* Ua = U + L->uoff[a];
    for (int li = 0; li < na; ++li) {
      float acc = 0.0f;
      for (int q = 0; q < ka; ++q) acc += Ua[(size_t)li * ka + q] * xc[L->coff[a] + q];
      x[L->arows[L->aptr[a] + li]] += acc;
    }
  }
  if (H->smoother == ORC_L1_JACOBI)
    l1_jacobi32(L, val, r, x);
  else
    gs_sweep32(H, l, val, r, x, 0);
  free(s);
  free(rc);
  free(xc);
}

/* ================================================================ API */

orc_hier* orc_create(int nl, const orc_level* lv, int smoother, int* status) {
  *status = 0;
  orc_hier* H = (orc_hier*)calloc(1, sizeof(orc_hier));
  H->nl = nl;
  H->smoother = smoother;
  H->lv = (orc_level*)malloc(sizeof(orc_level) * (size_t)nl);
  memcpy(H->lv, lv, sizeof(orc_level) * (size_t)nl);
  const orc_level* C = &lv[nl - 1];
  H->nL = C->n;
  H->Lc = (double*)calloc((size_t)C->n * (size_t)C->n, sizeof(double));
  for (int i = 0; i < C->n; ++i)
    for (int k = C->rowptr[i]; k < C->rowptr[i + 1]; ++k) H->Lc[(size_t)i * C->n + C->col[k]] += C->val[k];
  if (cholesky(H->Lc, C->n) != 0) *status = -3;
  H->val32 = (float**)calloc((size_t)nl, sizeof(float*));
  H->U32 = (float**)calloc((size_t)nl, sizeof(float*));
  for (int l = 0; l + 1 < nl; ++l) {
    const orc_level* L = &lv[l];
    const int nnz = L->rowptr[L->n];
    H->val32[l] = (float*)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
    for (int k = 0; k < nnz; ++k) H->val32[l][k] = (float)L->val[k];
    const int nu = L->uoff[L->nagg];
    H->U32[l] = (float*)malloc(sizeof(float) * (size_t)(nu > 0 ? nu : 1));
    for (int k = 0; k < nu; ++k) H->U32[l][k] = (float)L->U[k];
  }
  return H;
}

void orc_destroy(orc_hier* H) {
  if (!H) return;
  for (int l = 0; l < H->nl; ++l) {
    free(H->val32[l]);
    free(H->U32[l]);
  }
  free(H->val32);
  free(H->U32);
  free(H->Lc);
  free(H->lv);
  free(H);
}

void orc_vcycle(const orc_hier* H, const double* val0, const double* r, double* z) {
  vcycle(H, 0, val0, r, z);
}

void orc_vcycle32(const orc_hier* H, const float* val0_32, const float* r, float* z) {
  vcycle32(H, 0, val0_32, r, z);
}

/* Coarsest-level exact solve, exposed for tests. */
void orc_coarse_solve(const orc_hier* H, const double* r, double* z) { chol_solve(H->Lc, H->nL, r, z); }

/* One smoothing sweep on level l (forward != 0: forward), for tests. */
void orc_smooth(const orc_hier* H, int l, const double* r, double* x, int forward) {
  if (H->smoother == ORC_L1_JACOBI)
    l1_jacobi(&H->lv[l], H->lv[l].val, r, x);
  else
    gs_sweep(H, l, H->lv[l].val, r, x, forward);
}

/* The same sweep in binary32 on the level's binary32 values, for tests. */
void orc_smooth32(const orc_hier* H, int l, const float* r, float* x, int forward) {
  if (H->smoother == ORC_L1_JACOBI)
    l1_jacobi32(&H->lv[l], H->val32[l], r, x);
  else
    gs_sweep32(H, l, H->val32[l], r, x, forward);
}

void orc_spmv(int n, const int* rp, const int* ci, const double* v, const double* x, double* y) {
  csr_mv(n, rp, ci, v, x, y);
}

/*
 * Preconditioned CG (Section 5).  A is given by (rp, ci, v) with the
 * hierarchy's pattern at level 0; its values are also used for level-0
 * smoothing and the level-0 residual of the cycle (a near-by matrix, Section 1).
 * hist[0..nit] receives ||r_k|| / ||r_0||.  precond = 0 gives plain CG.
 * Returns 0 converged, 1 not converged, -5 breakdown (p^T A p <= 0).
 */
int orc_pcg(const orc_hier* H, int precond, int n, const int* rp, const int* ci, const double* v,
            const double* b, double* x, double tol, int maxit, double* hist, int* nit) {
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* z = (double*)malloc(sizeof(double) * (size_t)n);
  double* p = (double*)malloc(sizeof(double) * (size_t)n);
  double* q = (double*)malloc(sizeof(double) * (size_t)n);
  int status = 1;
  *nit = 0;
  csr_mv(n, rp, ci, v, x, q);
  for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
  const double r0 = sqrt(dotp(r, r, n));
  if (hist) hist[0] = 1.0;
  if (r0 == 0.0) {
    status = 0;
    goto done;
  }
  if (precond)
    vcycle(H, 0, v, r, z);
  else
    memcpy(z, r, sizeof(double) * (size_t)n);
  memcpy(p, z, sizeof(double) * (size_t)n);
  double rho = dotp(r, z, n);
  for (int k = 0; k < maxit; ++k) {
    csr_mv(n, rp, ci, v, p, q);
    const double pq = dotp(p, q, n);
    if (!(pq > 0.0)) {
      status = -5;
      break;
    }
    const double alpha = rho / pq;
    for (int i = 0; i < n; ++i) x[i] += alpha * p[i];
    for (int i = 0; i < n; ++i) r[i] -= alpha * q[i];
    *nit = k + 1;
    const double h = sqrt(dotp(r, r, n)) / r0;
    if (hist) hist[k + 1] = h;
    if (h <= tol) {
      status = 0;
      break;
    }
    if (precond)
      vcycle(H, 0, v, r, z);
    else
      memcpy(z, r, sizeof(double) * (size_t)n);
    const double rho_new = dotp(r, z, n);
    const double beta = rho_new / rho;
    rho = rho_new;
    for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
done:
  free(r);
  free(z);
  free(p);
  free(q);
  return status;
}

/*
 * Mixed precision: the V-cycle in binary32 (casts at its entry and exit),
 * everything else binary64.  Because the binary32 cycle is not an exactly
 * symmetric operator, CG uses the flexible beta that keeps p_{k+1} locally
 * A-orthogonal to p_k (Notay 2000): beta = z_{k+1}.(r_{k+1} - r_k) / (r_k . z_k),
 * evaluated with r_{k+1} - r_k = -alpha_k A p_k as beta = -alpha_k z_{k+1}.q_k / rho_k.
 * When the recursive residual
 * meets tol, the true residual b - A x is recomputed in binary64; if it does
 * not meet tol the iteration restarts from x (at most max_restarts times).
 * hist receives the recursive residual history (restarts continue it);
 * *nit counts all iterations, *restarts the restarts taken.  tol is relative
 * to the initial ||b - A x0||.
 */
int orc_pcg_mixed(const orc_hier* H, int n, const int* rp, const int* ci, const double* v,
                  const double* b, double* x, double tol, int maxit, int max_restarts, double* hist,
                  int* nit, double* true_rel, int* restarts) {
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* z = (double*)malloc(sizeof(double) * (size_t)n);
  double* p = (double*)malloc(sizeof(double) * (size_t)n);
  double* q = (double*)malloc(sizeof(double) * (size_t)n);
  float* r32 = (float*)malloc(sizeof(float) * (size_t)n);
  float* z32 = (float*)malloc(sizeof(float) * (size_t)n);
  float* v32 = (float*)malloc(sizeof(float) * (size_t)(rp[n] > 0 ? rp[n] : 1));
  for (int k = 0; k < rp[n]; ++k) v32[k] = (float)v[k];
  int status = 1, it = 0;
  *restarts = 0;
  csr_mv(n, rp, ci, v, x, q);
  for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
  const double r0 = sqrt(dotp(r, r, n));
  if (hist) hist[0] = 1.0;
  *true_rel = 0.0;
  if (r0 == 0.0) {
    status = 0;
    goto done;
  }
  for (int restart = 0; restart <= max_restarts && it < maxit; ++restart) {
    if (restart > 0) {
      *restarts = restart;
      csr_mv(n, rp, ci, v, x, q);
      for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
    }
    for (int i = 0; i < n; ++i) r32[i] = (float)r[i];
    vcycle32(H, 0, v32, r32, z32);
    for (int i = 0; i < n; ++i) z[i] = (double)z32[i];
    memcpy(p, z, sizeof(double) * (size_t)n);
    double rho = dotp(r, z, n);
    int met = 0;
    while (it < maxit) {
      csr_mv(n, rp, ci, v, p, q);
      const double pq = dotp(p, q, n);
      if (!(pq > 0.0)) {
        status = -5;
        goto done;
      }
      const double alpha = rho / pq;
      for (int i = 0; i < n; ++i) x[i] += alpha * p[i];
      for (int i = 0; i < n; ++i) r[i] -= alpha * q[i];
      ++it;
      const double h = sqrt(dotp(r, r, n)) / r0;
      if (hist) hist[it] = h;
      if (h <= tol) {
        met = 1;
        break;
      }
      for (int i = 0; i < n; ++i) r32[i] = (float)r[i];
      vcycle32(H, 0, v32, r32, z32);
      for (int i = 0; i < n; ++i) z[i] = (double)z32[i];
      const double beta = -alpha * dotp(z, q, n) / rho;
      rho = dotp(r, z, n);
      for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    /* true residual in binary64 */
    csr_mv(n, rp, ci, v, x, q);
    for (int i = 0; i < n; ++i) q[i] = b[i] - q[i];
    *true_rel = sqrt(dotp(q, q, n)) / r0;
    if (met && *true_rel <= tol) {
      status = 0;
      break;
    }
  }
done:
  *nit = it;
  free(r);
  free(z);
  free(p);
  free(q);
  free(r32);
  free(z32);
  free(v32);
  return status;
}

void orc_kcycle(const orc_hier* H, const double* val0, const double* r, double* z) {
  kcycle(H, 0, val0, r, z);
}

/*
 * CG preconditioned by the K-cycle.  The K-cycle is not a linear operator
 * (its inner coefficients depend on the residual), so CG takes the flexible
 * beta = -alpha_k z_{k+1}.q_k / rho_k (Notay 2000), as orc_pcg_mixed does.
 * Everything in binary64; stopping rule and history as orc_pcg.
 */
int orc_pcg_kcycle(const orc_hier* H, int n, const int* rp, const int* ci, const double* v, const double* b,
                   double* x, double tol, int maxit, double* hist, int* nit) {
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* z = (double*)malloc(sizeof(double) * (size_t)n);
  double* p = (double*)malloc(sizeof(double) * (size_t)n);
  double* q = (double*)malloc(sizeof(double) * (size_t)n);
  int status = 1;
  *nit = 0;
  csr_mv(n, rp, ci, v, x, q);
  for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
  const double r0 = sqrt(dotp(r, r, n));
  if (hist) hist[0] = 1.0;
  if (r0 == 0.0) {
    status = 0;
    goto done;
  }
  kcycle(H, 0, v, r, z);
  memcpy(p, z, sizeof(double) * (size_t)n);
  double rho = dotp(r, z, n);
  for (int k = 0; k < maxit; ++k) {
    csr_mv(n, rp, ci, v, p, q);
    const double pq = dotp(p, q, n);
    if (!(pq > 0.0)) {
      status = -5;
      break;
    }
    const double alpha = rho / pq;
    for (int i = 0; i < n; ++i) x[i] += alpha * p[i];
    for (int i = 0; i < n; ++i) r[i] -= alpha * q[i];
    *nit = k + 1;
    const double h = sqrt(dotp(r, r, n)) / r0;
    if (hist) hist[k + 1] = h;
    if (h <= tol) {
      status = 0;
      break;
    }
    kcycle(H, 0, v, r, z);
    const double beta = -alpha * dotp(z, q, n) / rho;
    rho = dotp(r, z, n);
    for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
done:
  free(r);
  free(z);
  free(p);
  free(q);
  return status;
}

/* ------------------------------------------------------ composite AMG */

/* z = B_k r with the V-cycle (kcyc == 0) or the K-cycle of hierarchy H; the
   level-0 values are v (every bootstrap hierarchy is built on the same A). */
static void component(const orc_hier* H, int kcyc, const double* v, const double* r, double* z) {
  if (kcyc)
    kcycle(H, 0, v, r, z);
  else
    vcycle(H, 0, v, r, z);
}

/* Index of the j-th factor of the symmetrized product, j = 0 .. 2r-1: the
   order 1, 2, .., r, r, .., 2, 1 (0-based). */
static int sym_index(int r, int j) { return j < r ? j : 2 * r - 1 - j; }

/*
 * z = B res for the symmetrized multiplicative composite of the r
 * hierarchies Hs (eq. 1.1 and Section 5 item (i)): its error propagator is
 * I - B A = (I - B_1 A)..(I - B_r A)(I - B_r A)..(I - B_1 A).  Starting from
 * z = 0, every factor k in the order 1, .., r, r, .., 1 takes
 * z <- z + B_k (res - A z), which multiplies the error A^{-1} res - z by
 * (I - B_k A); the factor applied first is the rightmost one.
 */
void orc_composite_apply(const orc_hier* const* Hs, int r, int kcyc, int n, const int* rp, const int* ci,
                         const double* v, const double* res, double* z) {
  double* t = (double*)malloc(sizeof(double) * (size_t)n);
  double* u = (double*)malloc(sizeof(double) * (size_t)n);
  for (int i = 0; i < n; ++i) z[i] = 0.0;
  for (int j = 0; j < 2 * r; ++j) {
    csr_mv(n, rp, ci, v, z, t);
    for (int i = 0; i < n; ++i) t[i] = res[i] - t[i];
    component(Hs[sym_index(r, j)], kcyc, v, t, u);
    for (int i = 0; i < n; ++i) z[i] += u[i];
  }
  free(t);
  free(u);
}

/*
 * The testing phase of Algorithm 1 with the symmetrized product: x <- E x,
 * E = (I - B_1 A)..(I - B_r A)(I - B_r A)..(I - B_1 A), nu times, from the
 * given x (every factor x <- x - B_k A x, rightmost first).  *rho receives
 * the convergence estimate ||x^nu||_A / ||x^{nu-1}||_A and x the new smooth
 * vector x^nu / ||x^nu||_A (left as x^nu when its A-norm is zero).
 */
void orc_composite_test(const orc_hier* const* Hs, int r, int kcyc, int nu, int n, const int* rp,
                        const int* ci, const double* v, double* x, double* rho) {
  double* t = (double*)malloc(sizeof(double) * (size_t)n);
  double* u = (double*)malloc(sizeof(double) * (size_t)n);
  double* prev = (double*)malloc(sizeof(double) * (size_t)n);
  for (int it = 0; it < nu; ++it) {
    memcpy(prev, x, sizeof(double) * (size_t)n);
    for (int j = 0; j < 2 * r; ++j) {
      csr_mv(n, rp, ci, v, x, t);
      component(Hs[sym_index(r, j)], kcyc, v, t, u);
      for (int i = 0; i < n; ++i) x[i] -= u[i];
    }
  }
  csr_mv(n, rp, ci, v, x, t);
  const double an = sqrt(fmax(0.0, dotp(x, t, n)));
  csr_mv(n, rp, ci, v, prev, t);
  const double ap = sqrt(fmax(0.0, dotp(prev, t, n)));
  *rho = (ap > 0.0) ? an / ap : 0.0;
  if (an > 0.0)
    for (int i = 0; i < n; ++i) x[i] /= an;
  free(t);
  free(u);
  free(prev);
}

/*
 * CG preconditioned by the composite AMG (the paper's original bootstrap
 * AMG, the b-it / b-ts comparison of Section 5).  With K-cycle components the
 * preconditioner is not linear, so CG takes the flexible beta
 * -alpha_k z_{k+1}.q_k / rho_k (Notay 2000) in both cases.  Stopping rule and
 * history as orc_pcg.
 */
int orc_pcg_composite(const orc_hier* const* Hs, int r, int kcyc, int n, const int* rp, const int* ci,
                      const double* v, const double* b, double* x, double tol, int maxit, double* hist, int* nit) {
  double* rr = (double*)malloc(sizeof(double) * (size_t)n);
  double* z = (double*)malloc(sizeof(double) * (size_t)n);
  double* p = (double*)malloc(sizeof(double) * (size_t)n);
  double* q = (double*)malloc(sizeof(double) * (size_t)n);
  int status = 1;
  *nit = 0;
  csr_mv(n, rp, ci, v, x, q);
  for (int i = 0; i < n; ++i) rr[i] = b[i] - q[i];
  const double r0 = sqrt(dotp(rr, rr, n));
  if (hist) hist[0] = 1.0;
  if (r0 == 0.0) {
    status = 0;
    goto done;
  }
  orc_composite_apply(Hs, r, kcyc, n, rp, ci, v, rr, z);
  memcpy(p, z, sizeof(double) * (size_t)n);
  double rho = dotp(rr, z, n);
  for (int k = 0; k < maxit; ++k) {
    csr_mv(n, rp, ci, v, p, q);
    const double pq = dotp(p, q, n);
    if (!(pq > 0.0)) {
      status = -5;
      break;
    }
    const double alpha = rho / pq;
    for (int i = 0; i < n; ++i) x[i] += alpha * p[i];
    for (int i = 0; i < n; ++i) rr[i] -= alpha * q[i];
    *nit = k + 1;
    const double h = sqrt(dotp(rr, rr, n)) / r0;
    if (hist) hist[k + 1] = h;
    if (h <= tol) {
      status = 0;
      break;
    }
    orc_composite_apply(Hs, r, kcyc, n, rp, ci, v, rr, z);
    const double beta = -alpha * dotp(z, q, n) / rho;
    rho = dotp(rr, z, n);
    for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
done:
  free(rr);
  free(z);
  free(p);
  free(q);
  return status;
}

/* dL/da_ij = -lambda_i x_j for every stored entry (i, j) of the CSR pattern. */
void orc_grad_coeffs(int n, const int* rp, const int* ci, const double* lambda, const double* x,
                     double* dval) {
  for (int i = 0; i < n; ++i)
    for (int k = rp[i]; k < rp[i + 1]; ++k) dval[k] = -lambda[i] * x[ci[k]];
}
