/*
 * Reference oracle for the multi-time-step (MTS) coupling of bond-based
 * peridynamics and finite elements in the Arlequin framework
 * (Zhong, Han, Du, Guo, arXiv 2403.03605).
 *
 * TEST INFRASTRUCTURE ONLY: plain FP64 loops, no blocking, no reordering.
 * Each function names the passage of the paper it follows.  Where the paper is
 * silent the reading taken is stated next to the code, numbered R1, R2, ...
 * Built with -O2 -ffp-contract=off so that every expression is evaluated
 * exactly as written.
 */
#include "mts_oracle.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static __thread char g_err[512];

static void set_err(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

const char *orc_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------- */
/* Neighbourhood H_delta(x) = {x' : |x' - x| <= delta}  (Sec. 2.1)            */
/* ------------------------------------------------------------------------- */

/* Squared distance, evaluated left to right: ((dx*dx + dy*dy) + dz*dz). */
static double dist2(int dim, const double *a, const double *b) {
  double d0 = b[0] - a[0];
  double d1 = b[1] - a[1];
  double r2 = d0 * d0 + d1 * d1;
  if (dim == 3) {
    double d2 = b[2] - a[2];
    r2 = r2 + d2 * d2;
  }
  return r2;
}

int64_t orc_neighbors_brute(int dim, int64_t n, const double *x, double delta,
                            int64_t *row_ptr, int32_t *col, int64_t cap) {
  double d2 = delta * delta;
  int64_t nnz = 0;
  row_ptr[0] = 0;
  for (int64_t i = 0; i < n; i++) {
    for (int64_t k = 0; k < n; k++) {
      if (k == i) continue;
      if (dist2(dim, x + i * dim, x + k * dim) <= d2) {
        if (nnz >= cap) return -1;
        col[nnz++] = (int32_t)k;
      }
    }
    row_ptr[i + 1] = nnz;
  }
  return nnz;
}

static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

/* Same set as the brute-force search, found through bins of side delta. */
int64_t orc_neighbors_grid(int dim, int64_t n, const double *x, double delta,
                           int64_t *row_ptr, int32_t *col, int64_t cap) {
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  int64_t nb[3] = {1, 1, 1};
  for (int a = 0; a < dim; a++) {
    lo[a] = hi[a] = x[a];
    for (int64_t i = 0; i < n; i++) {
      if (x[i * dim + a] < lo[a]) lo[a] = x[i * dim + a];
      if (x[i * dim + a] > hi[a]) hi[a] = x[i * dim + a];
    }
    nb[a] = (int64_t)floor((hi[a] - lo[a]) / delta) + 1;
  }
  int64_t nbins = nb[0] * nb[1] * nb[2];
  int64_t *bin_of = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *start = calloc((size_t)nbins + 1, sizeof(int64_t));
  int64_t *items = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *fill = calloc((size_t)nbins, sizeof(int64_t));
  int64_t *cand = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!bin_of || !start || !items || !fill || !cand) {
    free(bin_of); free(start); free(items); free(fill); free(cand);
    return -1;
  }
  for (int64_t i = 0; i < n; i++) {
    int64_t b[3] = {0, 0, 0};
    for (int a = 0; a < dim; a++) {
      b[a] = (int64_t)floor((x[i * dim + a] - lo[a]) / delta);
      if (b[a] >= nb[a]) b[a] = nb[a] - 1;
      if (b[a] < 0) b[a] = 0;
    }
    bin_of[i] = (b[2] * nb[1] + b[1]) * nb[0] + b[0];
    start[bin_of[i] + 1]++;
  }
  for (int64_t q = 0; q < nbins; q++) start[q + 1] += start[q];
  for (int64_t i = 0; i < n; i++) items[start[bin_of[i]] + fill[bin_of[i]]++] = i;

  double d2 = delta * delta;
  int64_t nnz = 0;
  row_ptr[0] = 0;
  for (int64_t i = 0; i < n; i++) {
    int64_t b = bin_of[i];
    int64_t bx = b % nb[0], by = (b / nb[0]) % nb[1], bz = b / (nb[0] * nb[1]);
    int64_t nc = 0;
    for (int64_t dz = -1; dz <= 1; dz++)
      for (int64_t dy = -1; dy <= 1; dy++)
        for (int64_t dxx = -1; dxx <= 1; dxx++) {
          int64_t cx = bx + dxx, cy = by + dy, cz = bz + dz;
          if (cx < 0 || cy < 0 || cz < 0 || cx >= nb[0] || cy >= nb[1] || cz >= nb[2]) continue;
          int64_t q = (cz * nb[1] + cy) * nb[0] + cx;
          for (int64_t t = start[q]; t < start[q + 1]; t++) cand[nc++] = items[t];
        }
    qsort(cand, (size_t)nc, sizeof(int64_t), cmp_i64);
    for (int64_t t = 0; t < nc; t++) {
      int64_t k = cand[t];
      if (k == i) continue;
      if (dist2(dim, x + i * dim, x + k * dim) <= d2) {
        if (nnz >= cap) {
          nnz = -1;
          goto done;
        }
        col[nnz++] = (int32_t)k;
      }
    }
    row_ptr[i + 1] = nnz;
  }
done:
  free(bin_of); free(start); free(items); free(fill); free(cand);
  return nnz;
}

/* int_0^delta r^n exp(-r/l) dr = l^(n+1) n! (1 - exp(-delta/l) sum_{k<=n} (delta/l)^k / k!) */
double orc_exp_moment(int n, double delta, double l) {
  double t = delta / l, term = 1.0, sum = 1.0, fact = 1.0;
  for (int k = 1; k <= n; k++) {
    term = term * t / (double)k;
    sum = sum + term;
    fact = fact * (double)k;
  }
  return pow(l, (double)(n + 1)) * fact * (1.0 - exp(-t) * sum);
}

/* ------------------------------------------------------------------------- */
/* Solver state                                                              */
/* ------------------------------------------------------------------------- */
struct orc_solver {
  orc_problem p;
  int dim;
  int64_t N;
  double *x;
  double delta, d2, V, VV, c0, lexp, scrit, nu;
  double dtP, hdtP, hdt2P, dtF, hdtF, hdt2F;
  double o2lo[3], o2hi[3];
  /* bonds */
  int64_t *rp;
  int32_t *col;
  uint8_t *mu, *musnap;
  int64_t nnz;
  /* PD nodes */
  double *alpha, *mP, *uP, *vP, *aP, *PP;
  /* FE */
  int nen, ngp, nstr;
  int64_t nfe, ne, fgrid[3];
  int32_t *conn;
  uint8_t *eact, *nact, *bc;
  double *xF, *gpa, *mF, *uF, *vF, *aF, *PF;
  double D[6][6];
  double Ngp[8][8], dNgp[8][8][3]; /* per gauss point, per local node */
  double detJ;
  /* implicit FE (Newmark beta > 0): Cholesky factor of the dense system matrix
   * A = M + beta dt^2 K over all FE dofs (identity on prescribed and inactive dofs) */
  double beta;
  double *LA;
  double *LP;                 /* implicit PD: Cholesky factor of M + beta dt^2 K_PD (N dim)^2 */
  double betaP;
  double *febuf;              /* per-element internal forces of orc_fe_force (ne * nen * dim) */
  /* coupling */
  int64_t nc, nl;
  int64_t *cn, *cel, *cidx;
  double *cw;
  double *H, *L, *lam0;
  int64_t *ycnt;
  int64_t **ynode;
  double **yval;
  uint8_t *region;
  int64_t nregion;
  /* counters */
  int64_t pd_steps, macro_steps, nrebuild, nbroken;
};

static void *xcalloc(size_t n, size_t sz) {
  void *q = calloc(n ? n : 1, sz);
  if (!q) set_err("out of memory (%zu x %zu)", n, sz);
  return q;
}

/* Arlequin weight alpha(x) (Eq. 17-18, weight functions of Sec. 3.2).
 * l1 is the L-infinity distance from x to the PD-only box Omega^2 (reading R9);
 * alpha = 1 once l1 >= l^O, i.e. outside the PD box. */
static double alpha_at(const orc_solver *s, const double *x) {
  if (s->p.mode == ORC_PURE_PD) return 0.0;
  if (s->p.mode == ORC_PURE_FE) return 1.0;
  double l1 = 0.0;
  for (int a = 0; a < s->dim; a++) {
    double d = s->o2lo[a] - x[a];
    double e = x[a] - s->o2hi[a];
    if (e > d) d = e;
    if (d > l1) l1 = d;
  }
  double lO = s->p.overlap;
  if (l1 >= lO) return 1.0;
  if (l1 <= 0.0) return 0.0;
  double t = l1 / lO;
  if (s->p.weight_kind == ORC_W_LINEAR) return t;
  if (s->p.weight_kind == ORC_W_CONSTANT) return 0.5;
  return t * t * t;
}

/* Micromodulus c(|xi|) of Eq. 2 (reading R2: PMB-equivalent c0/r^3, or the
 * exponential kernel of Sec. 3.2 / Sec. 3.3). */
static double cfun(const orc_solver *s, double r) {
  if (s->p.kernel == ORC_K_EXP) return s->c0 * exp(-r / s->lexp);
  return s->c0 / (r * r * r);
}

/* Pre-crack (reading R19): bond i-k is cut iff it crosses the horizontal
 * segment y = yc, x_start <= x* <= x_end.  x* is computed from the endpoint
 * with the smaller id so both directions of a bond take the same decision. */
static int crosses_crack(const orc_solver *s, int64_t i, int64_t k) {
  if (s->dim != 2) return 0;
  int64_t p = i < k ? i : k, q = i < k ? k : i;
  const double *xp = s->x + 2 * p, *xq = s->x + 2 * q;
  for (int c = 0; c < s->p.n_cracks; c++) {
    double yc = s->p.cracks[c][0];
    if ((xp[1] - yc) * (xq[1] - yc) < 0.0) {
      double xs = xp[0] + (yc - xp[1]) * (xq[0] - xp[0]) / (xq[1] - xp[1]);
      if (xs >= s->p.cracks[c][1] && xs <= s->p.cracks[c][2]) return 1;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Finite elements: Q4 / Hex8, 2x2(x2) Gauss, alpha at each Gauss point       */
/* (Eq. 24-27, Eq. 34, readings R10, R11, R20)                               */
/* ------------------------------------------------------------------------- */
static const double q4_nat[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
static const double h8_nat[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                    {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

static double shape(int dim, int a, const double *xi) {
  if (dim == 2) return 0.25 * (1.0 + q4_nat[a][0] * xi[0]) * (1.0 + q4_nat[a][1] * xi[1]);
  return 0.125 * (1.0 + h8_nat[a][0] * xi[0]) * (1.0 + h8_nat[a][1] * xi[1]) *
         (1.0 + h8_nat[a][2] * xi[2]);
}

/* d N_a / d x (physical), square elements of side h. */
static void dshape(int dim, int a, const double *xi, double h, double *out) {
  double g = 2.0 / h;
  if (dim == 2) {
    out[0] = g * 0.25 * q4_nat[a][0] * (1.0 + q4_nat[a][1] * xi[1]);
    out[1] = g * 0.25 * q4_nat[a][1] * (1.0 + q4_nat[a][0] * xi[0]);
  } else {
    out[0] = g * 0.125 * h8_nat[a][0] * (1.0 + h8_nat[a][1] * xi[1]) * (1.0 + h8_nat[a][2] * xi[2]);
    out[1] = g * 0.125 * h8_nat[a][1] * (1.0 + h8_nat[a][0] * xi[0]) * (1.0 + h8_nat[a][2] * xi[2]);
    out[2] = g * 0.125 * h8_nat[a][2] * (1.0 + h8_nat[a][0] * xi[0]) * (1.0 + h8_nat[a][1] * xi[1]);
  }
}

static void gauss_point(int dim, int g, double *xi) {
  double q = 1.0 / sqrt(3.0);
  xi[0] = (g & 1) ? q : -q;
  xi[1] = (g & 2) ? q : -q;
  if (dim == 3) xi[2] = (g & 4) ? q : -q;
}

/* Strain of one element at one Gauss point: eps = B u_e (engineering shear). */
static void strain(const orc_solver *s, int g, const double *ue, double *eps) {
  int dim = s->dim;
  for (int r = 0; r < s->nstr; r++) eps[r] = 0.0;
  for (int a = 0; a < s->nen; a++) {
    const double *dN = s->dNgp[g][a];
    const double *u = ue + a * dim;
    if (dim == 2) {
      eps[0] += dN[0] * u[0];
      eps[1] += dN[1] * u[1];
      eps[2] += dN[1] * u[0] + dN[0] * u[1];
    } else {
      eps[0] += dN[0] * u[0];
      eps[1] += dN[1] * u[1];
      eps[2] += dN[2] * u[2];
      eps[3] += dN[1] * u[0] + dN[0] * u[1];
      eps[4] += dN[2] * u[1] + dN[1] * u[2];
      eps[5] += dN[2] * u[0] + dN[0] * u[2];
    }
  }
}

/* f_e += scale * B^T sig */
static void btsig(const orc_solver *s, int g, const double *sig, double scale, double *fe) {
  int dim = s->dim;
  for (int a = 0; a < s->nen; a++) {
    const double *dN = s->dNgp[g][a];
    double *f = fe + a * dim;
    if (dim == 2) {
      f[0] += scale * (dN[0] * sig[0] + dN[1] * sig[2]);
      f[1] += scale * (dN[1] * sig[1] + dN[0] * sig[2]);
    } else {
      f[0] += scale * (dN[0] * sig[0] + dN[1] * sig[3] + dN[2] * sig[5]);
      f[1] += scale * (dN[1] * sig[1] + dN[0] * sig[3] + dN[2] * sig[4]);
      f[2] += scale * (dN[2] * sig[2] + dN[1] * sig[4] + dN[0] * sig[5]);
    }
  }
}

/* Internal force K_F u = sum_e sum_gp alpha B^T D B u detJ t  (Eq. 27, Eq. 34). */
int orc_fe_force(orc_solver *s, const double *u, double *f) {
  int dim = s->dim;
  int nd = s->nen * dim;
  if (!s->febuf) {
    s->febuf = xcalloc((size_t)(s->ne * nd), sizeof(double));
    if (!s->febuf) return -1;
  }
  /* element forces are independent, so an OpenMP build computes them in
   * parallel; the scatter below adds them in ascending element order either way */
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < s->ne; e++) {
    double ue[24], eps[6], sig[6];
    double *fe = s->febuf + e * nd;
    for (int t = 0; t < nd; t++) fe[t] = 0.0;
    if (!s->eact[e]) continue;
    for (int a = 0; a < s->nen; a++)
      for (int d = 0; d < dim; d++) ue[a * dim + d] = u[(int64_t)s->conn[e * s->nen + a] * dim + d];
    for (int g = 0; g < s->ngp; g++) {
      double al = s->gpa[e * s->ngp + g];
      if (al == 0.0) continue;
      strain(s, g, ue, eps);
      for (int r = 0; r < s->nstr; r++) {
        sig[r] = 0.0;
        for (int c = 0; c < s->nstr; c++) sig[r] += s->D[r][c] * eps[c];
      }
      btsig(s, g, sig, al * s->detJ * s->p.thickness, fe);
    }
  }
  memset(f, 0, sizeof(double) * (size_t)(s->nfe * dim));
  for (int64_t e = 0; e < s->ne; e++) {
    if (!s->eact[e]) continue;
    const double *fe = s->febuf + e * nd;
    for (int a = 0; a < s->nen; a++)
      for (int d = 0; d < dim; d++) f[(int64_t)s->conn[e * s->nen + a] * dim + d] += fe[a * dim + d];
  }
  return 0;
}

/* Free (unprescribed, active) FE dof? */
static int fe_free_dof(const orc_solver *s, int64_t t) {
  return s->nact[t / s->dim] && !s->bc[t];
}

/* Implicit FE (Newmark, Eq. 38 with beta > 0): A = M + beta dt_FE^2 K on the
 * free dofs, the identity on prescribed and inactive ones (their acceleration
 * is zero), assembled column by column from the internal force and factored
 * (Cholesky, A = L L^T). */
static int build_fe_implicit(orc_solver *s) {
  int64_t nF = s->nfe * s->dim;
  double c = s->beta * s->dtF * s->dtF;
  double *A = xcalloc((size_t)(nF * nF), sizeof(double));
  double *e = xcalloc((size_t)nF, sizeof(double));
  double *f = xcalloc((size_t)nF, sizeof(double));
  s->LA = A;
  if (!A || !e || !f) { free(e); free(f); return -1; }
  for (int64_t j = 0; j < nF; j++) {
    if (!fe_free_dof(s, j)) {
      A[j * nF + j] = 1.0;
      continue;
    }
    e[j] = 1.0;
    orc_fe_force(s, e, f); /* column j of K */
    e[j] = 0.0;
    for (int64_t i = 0; i < nF; i++)
      if (fe_free_dof(s, i)) A[i * nF + j] = c * f[i];
    A[j * nF + j] += s->mF[j / s->dim];
  }
  free(e);
  free(f);
  for (int64_t j = 0; j < nF; j++) {
    double d = A[j * nF + j];
    for (int64_t k = 0; k < j; k++) d -= A[j * nF + k] * A[j * nF + k];
    if (!(d > 0.0)) { set_err("implicit FE matrix not positive definite at row %lld", (long long)j); return -1; }
    double ljj = sqrt(d);
    A[j * nF + j] = ljj;
    for (int64_t i = j + 1; i < nF; i++) {
      double t = A[i * nF + j];
      for (int64_t k = 0; k < j; k++) t -= A[i * nF + k] * A[j * nF + k];
      A[i * nF + j] = t / ljj;
    }
  }
  return 0;
}

/* x = A^-1 b through the Cholesky factor (x and b may alias). */
static void fe_solve(const orc_solver *s, const double *b, double *x) {
  int64_t nF = s->nfe * s->dim;
  const double *L = s->LA;
  for (int64_t i = 0; i < nF; i++) {
    double t = b[i];
    for (int64_t k = 0; k < i; k++) t -= L[i * nF + k] * x[k];
    x[i] = t / L[i * nF + i];
  }
  for (int64_t i = nF - 1; i >= 0; i--) {
    double t = x[i];
    for (int64_t k = i + 1; k < nF; k++) t -= L[k * nF + i] * x[k];
    x[i] = t / L[i * nF + i];
  }
}

static int build_fe(orc_solver *s) {
  int dim = s->dim;
  const orc_problem *p = &s->p;
  double h = p->fe_h;
  s->nen = dim == 2 ? 4 : 8;
  s->ngp = s->nen;
  s->nstr = dim == 2 ? 3 : 6;
  s->detJ = dim == 2 ? (h / 2) * (h / 2) : (h / 2) * (h / 2) * (h / 2);
  for (int g = 0; g < s->ngp; g++) {
    double xi[3];
    gauss_point(dim, g, xi);
    for (int a = 0; a < s->nen; a++) {
      s->Ngp[g][a] = shape(dim, a, xi);
      dshape(dim, a, xi, h, s->dNgp[g][a]);
    }
  }
  /* Hooke's law (Eq. 9): plane stress in 2D, isotropic in 3D. */
  memset(s->D, 0, sizeof s->D);
  double E = p->E, nu = s->nu;
  if (dim == 2) {
    double k = E / (1.0 - nu * nu);
    s->D[0][0] = k; s->D[0][1] = k * nu;
    s->D[1][0] = k * nu; s->D[1][1] = k;
    s->D[2][2] = k * (1.0 - nu) / 2.0;
  } else {
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    double mu = E / (2.0 * (1.0 + nu));
    for (int r = 0; r < 3; r++)
      for (int c = 0; c < 3; c++) s->D[r][c] = lam + (r == c ? 2.0 * mu : 0.0);
    s->D[3][3] = s->D[4][4] = s->D[5][5] = mu;
  }
  int64_t nx = p->fe_n[0], ny = p->fe_n[1], nz = dim == 3 ? p->fe_n[2] : 0;
  s->fgrid[0] = nx + 1; s->fgrid[1] = ny + 1; s->fgrid[2] = dim == 3 ? nz + 1 : 1;
  int64_t ngrid = s->fgrid[0] * s->fgrid[1] * s->fgrid[2];
  s->ne = nx * ny * (dim == 3 ? nz : 1);

  /* slit nodes (reading R20): duplicate grid nodes on each crack line with
   * x_start <= x < x_end; elements above the line use the copy. */
  int64_t *dup = xcalloc((size_t)ngrid, sizeof(int64_t));
  if (!dup) return -1;
  int64_t nextra = 0;
  int64_t jc[8];
  for (int c = 0; c < p->n_cracks && dim == 2; c++) {
    double yc = p->cracks[c][0];
    double jf = (yc - p->dom_lo[1]) / h;
    jc[c] = (int64_t)llround(jf);
    if (fabs(jf - (double)jc[c]) > 1e-6 || jc[c] <= 0 || jc[c] >= ny) {
      set_err("crack line y=%g is not an interior FE node line", yc);
      free(dup);
      return -1;
    }
    for (int64_t i = 0; i <= nx; i++) {
      double xn = p->dom_lo[0] + (double)i * h;
      if (xn >= p->cracks[c][1] - 1e-9 * h && xn < p->cracks[c][2] - 1e-9 * h) {
        int64_t g = jc[c] * (nx + 1) + i;
        if (!dup[g]) dup[g] = ngrid + (++nextra) - 1 + 1; /* store id+1 */
      }
    }
  }
  s->nfe = ngrid + nextra;
  s->conn = xcalloc((size_t)(s->ne * s->nen), sizeof(int32_t));
  s->xF = xcalloc((size_t)(s->nfe * dim), sizeof(double));
  s->eact = xcalloc((size_t)s->ne, 1);
  s->nact = xcalloc((size_t)s->nfe, 1);
  s->gpa = xcalloc((size_t)(s->ne * s->ngp), sizeof(double));
  s->mF = xcalloc((size_t)s->nfe, sizeof(double));
  s->uF = xcalloc((size_t)(s->nfe * dim), sizeof(double));
  s->vF = xcalloc((size_t)(s->nfe * dim), sizeof(double));
  s->aF = xcalloc((size_t)(s->nfe * dim), sizeof(double));
  s->PF = xcalloc((size_t)(s->nfe * dim), sizeof(double));
  s->bc = xcalloc((size_t)(s->nfe * dim), 1);
  if (!s->conn || !s->xF || !s->eact || !s->nact || !s->gpa || !s->mF || !s->uF || !s->vF ||
      !s->aF || !s->PF || !s->bc) {
    free(dup);
    return -1;
  }
  for (int64_t k = 0; k < s->fgrid[2]; k++)
    for (int64_t j = 0; j < s->fgrid[1]; j++)
      for (int64_t i = 0; i < s->fgrid[0]; i++) {
        int64_t g = (k * s->fgrid[1] + j) * s->fgrid[0] + i;
        s->xF[g * dim + 0] = p->dom_lo[0] + (double)i * h;
        s->xF[g * dim + 1] = p->dom_lo[1] + (double)j * h;
        if (dim == 3) s->xF[g * dim + 2] = p->dom_lo[2] + (double)k * h;
        if (dup[g]) {
          int64_t q = dup[g] - 1;
          for (int d = 0; d < dim; d++) s->xF[q * dim + d] = s->xF[g * dim + d];
        }
      }
  for (int64_t ez = 0; ez < (dim == 3 ? nz : 1); ez++)
    for (int64_t ey = 0; ey < ny; ey++)
      for (int64_t ex = 0; ex < nx; ex++) {
        int64_t e = (ez * ny + ey) * nx + ex;
        for (int a = 0; a < s->nen; a++) {
          const double *na = dim == 2 ? q4_nat[a] : h8_nat[a];
          int64_t i = ex + (na[0] > 0), j = ey + (na[1] > 0), k = dim == 3 ? ez + (na[2] > 0) : 0;
          int64_t g = (k * s->fgrid[1] + j) * s->fgrid[0] + i;
          int64_t node = g;
          /* bottom nodes of an element whose lower edge lies on a slit row */
          if (dup[g] && na[1] < 0) node = dup[g] - 1;
          s->conn[e * s->nen + a] = (int32_t)node;
        }
        double x0[3] = {p->dom_lo[0] + (double)ex * h, p->dom_lo[1] + (double)ey * h,
                        dim == 3 ? p->dom_lo[2] + (double)ez * h : 0.0};
        int act = 0;
        for (int g = 0; g < s->ngp; g++) {
          double xi[3], xg[3];
          gauss_point(dim, g, xi);
          for (int d = 0; d < dim; d++) xg[d] = x0[d] + (xi[d] + 1.0) * (h / 2.0);
          double al = alpha_at(s, xg);
          s->gpa[e * s->ngp + g] = al;
          if (al > 0.0) act = 1;
        }
        s->eact[e] = (uint8_t)act;
      }
  free(dup);
  /* Lumped (row-sum) weighted mass (Eq. 34, reading R10). */
  for (int64_t e = 0; e < s->ne; e++) {
    if (!s->eact[e]) continue;
    for (int g = 0; g < s->ngp; g++) {
      double al = s->gpa[e * s->ngp + g];
      for (int a = 0; a < s->nen; a++) {
        int64_t n = s->conn[e * s->nen + a];
        s->mF[n] += al * p->rho * s->Ngp[g][a] * s->detJ * p->thickness;
        s->nact[n] = 1;
      }
    }
  }
  /* Tractions on the faces y = dom_lo (outward -y) and y = dom_hi (+y), weighted
   * by alpha (Eq. 34 P^FE), 2-point Gauss per edge direction. */
  if (p->traction != 0.0) {
    double q = 1.0 / sqrt(3.0);
    for (int64_t ez = 0; ez < (dim == 3 ? nz : 1); ez++)
      for (int64_t ex = 0; ex < nx; ex++)
        for (int side = 0; side < 2; side++) {
          int64_t ey = side == 0 ? 0 : ny - 1;
          int64_t e = (ez * ny + ey) * nx + ex;
          if (!s->eact[e]) continue;
          double eta = side == 0 ? -1.0 : 1.0;
          double ty = side == 0 ? -p->traction : p->traction;
          int ngp2 = dim == 2 ? 2 : 4;
          for (int g = 0; g < ngp2; g++) {
            double xi[3] = {(g & 1) ? q : -q, eta, (g & 2) ? q : -q};
            double xg[3] = {p->dom_lo[0] + (double)ex * h + (xi[0] + 1.0) * (h / 2.0),
                            side == 0 ? p->dom_lo[1] : p->dom_hi[1],
                            dim == 3 ? p->dom_lo[2] + (double)ez * h + (xi[2] + 1.0) * (h / 2.0) : 0.0};
            double al = alpha_at(s, xg);
            double jac = dim == 2 ? h / 2.0 : (h / 2.0) * (h / 2.0);
            for (int a = 0; a < s->nen; a++) {
              double Na = shape(dim, a, xi);
              if (Na == 0.0) continue;
              int64_t n = s->conn[e * s->nen + a];
              s->PF[n * dim + 1] += al * Na * ty * jac * p->thickness;
            }
          }
        }
  }
  /* Uniform traction (+x) on the face x = dom_hi, alpha-weighted as above: the
   * end load of the beam of Sec. 3.2. */
  if (p->traction_x != 0.0) {
    double q = 1.0 / sqrt(3.0);
    int64_t ex = nx - 1;
    for (int64_t ez = 0; ez < (dim == 3 ? nz : 1); ez++)
      for (int64_t ey = 0; ey < ny; ey++) {
        int64_t e = (ez * ny + ey) * nx + ex;
        if (!s->eact[e]) continue;
        int ngp2 = dim == 2 ? 2 : 4;
        for (int g = 0; g < ngp2; g++) {
          double xi[3] = {1.0, (g & 1) ? q : -q, (g & 2) ? q : -q};
          double xg[3] = {p->dom_hi[0], p->dom_lo[1] + (double)ey * h + (xi[1] + 1.0) * (h / 2.0),
                          dim == 3 ? p->dom_lo[2] + (double)ez * h + (xi[2] + 1.0) * (h / 2.0) : 0.0};
          double al = alpha_at(s, xg);
          double jac = dim == 2 ? h / 2.0 : (h / 2.0) * (h / 2.0);
          for (int a = 0; a < s->nen; a++) {
            double Na = shape(dim, a, xi);
            if (Na == 0.0) continue;
            int64_t n = s->conn[e * s->nen + a];
            s->PF[n * dim] += al * Na * p->traction_x * jac * p->thickness;
          }
        }
      }
  }
  /* Clamped face x = dom_lo: every component held at zero (the beam's fixed
   * end); with vel_bc = 0 a flagged dof keeps u = v = a = 0. */
  if (p->clamp_x0) {
    for (int64_t n = 0; n < s->nfe; n++)
      if (s->nact[n] && fabs(s->xF[n * dim] - p->dom_lo[0]) < 1e-9 * h)
        for (int d = 0; d < dim; d++) s->bc[n * dim + d] = 1;
  }
  /* Prescribed velocity on the face x = dom_lo (x component). */
  if (p->vel_bc != 0.0) {
    for (int64_t n = 0; n < s->nfe; n++)
      if (s->nact[n] && fabs(s->xF[n * dim] - p->dom_lo[0]) < 1e-9 * h) {
        s->bc[n * dim] = 1;
        s->vF[n * dim] = p->vel_bc;
      }
  }
  for (int64_t n = 0; n < s->nfe; n++)
    if (s->nact[n])
      for (int d = 0; d < dim; d++)
        if (!s->bc[n * dim + d]) s->aF[n * dim + d] = s->PF[n * dim + d] / s->mF[n];
  return 0;
}

/* ------------------------------------------------------------------------- */
/* PD bond pass: Eq. 2 force, Eq. 3 stretch, Eq. 4 bond state                */
/* ------------------------------------------------------------------------- */

/* Force on node i from its family for displacement u.  brk: apply the
 * critical-stretch test first (reading R6: break first, inclusive s >= s_crit).
 * mu: bond states used (and updated when brk). Returns number of new breaks. */
static int64_t node_force(orc_solver *s, int64_t i, const double *u, uint8_t *mu, int brk,
                          double *F) {
  int dim = s->dim;
  const double *xi_ = s->x + i * dim, *ui = u + i * dim;
  int64_t broke = 0;
  F[0] = F[1] = F[2] = 0.0;
  for (int64_t t = s->rp[i]; t < s->rp[i + 1]; t++) {
    int64_t k = s->col[t];
    const double *xk = s->x + k * dim, *uk = u + k * dim;
    double xi[3] = {0, 0, 0}, eta[3] = {0, 0, 0};
    for (int d = 0; d < dim; d++) {
      xi[d] = xk[d] - xi_[d];
      eta[d] = uk[d] - ui[d];
    }
    if (brk && mu[t]) {
      double y[3] = {0, 0, 0};
      for (int d = 0; d < dim; d++) y[d] = xi[d] + eta[d];
      double r2 = xi[0] * xi[0] + xi[1] * xi[1];
      double y2 = y[0] * y[0] + y[1] * y[1];
      if (dim == 3) {
        r2 = r2 + xi[2] * xi[2];
        y2 = y2 + y[2] * y[2];
      }
      double r = sqrt(r2), ly = sqrt(y2);
      double st = (ly - r) / r;                 /* Eq. 3 */
      if (st >= s->scrit) {                      /* Eq. 4 */
        mu[t] = 0;
        broke++;
      }
    }
    if (!mu[t]) continue;
    double r2 = xi[0] * xi[0] + xi[1] * xi[1];
    double xe = xi[0] * eta[0] + xi[1] * eta[1];
    if (dim == 3) {
      r2 = r2 + xi[2] * xi[2];
      xe = xe + xi[2] * eta[2];
    }
    double r = sqrt(r2);
    double w = 1.0 - 0.5 * (s->alpha[i] + s->alpha[k]); /* reading R8 */
    double tt = ((w * cfun(s, r)) * xe) * s->VV;       /* Eq. 2, times V_i V_k */
    for (int d = 0; d < dim; d++) F[d] += tt * xi[d];
  }
  return broke;
}

int orc_pd_force(orc_solver *s, const double *u, double *f) {
  double F[3];
  for (int64_t i = 0; i < s->N; i++) {
    node_force(s, i, u, s->mu, 0, F);
    for (int d = 0; d < s->dim; d++) f[i * s->dim + d] = F[d];
  }
  return 0;
}

/* Deformation energy 1/4 sum_i sum_k mu w c (xi.eta)^2 V_i V_k (Eq. 6-7). */
double orc_pd_energy(orc_solver *s, const double *u) {
  int dim = s->dim;
  double E = 0.0;
  for (int64_t i = 0; i < s->N; i++)
    for (int64_t t = s->rp[i]; t < s->rp[i + 1]; t++) {
      if (!s->mu[t]) continue;
      int64_t k = s->col[t];
      double r2 = 0.0, xe = 0.0;
      for (int d = 0; d < dim; d++) {
        double xi = s->x[k * dim + d] - s->x[i * dim + d];
        double eta = u[k * dim + d] - u[i * dim + d];
        r2 += xi * xi;
        xe += xi * eta;
      }
      double w = 1.0 - 0.5 * (s->alpha[i] + s->alpha[k]);
      E += 0.25 * w * cfun(s, sqrt(r2)) * xe * xe * s->VV;
    }
  return E;
}

/* ------------------------------------------------------------------------- */
/* Unit-load responses Y^PD and the multiplier matrix H  (eq. unit, Eq. 49)   */
/* ------------------------------------------------------------------------- */
static void free_y(orc_solver *s) {
  if (s->ynode)
    for (int64_t c = 0; c < s->nl; c++) {
      free(s->ynode[c]);
      free(s->yval[c]);
    }
  free(s->ynode); free(s->yval); free(s->ycnt);
  s->ynode = NULL; s->yval = NULL; s->ycnt = NULL;
}

/* Link problem (Eq. 48b) for a unit multiplier on constraint dof c, run for m
 * substeps with bond states musnap and no breaking (Sec. 2.5, note on broken bonds).  The response is
 * exactly zero beyond (m-1) horizons of the loaded node, so only nodes of that
 * ball are stepped; all others keep their zero state. */
static int build_y(orc_solver *s) {
  int dim = s->dim;
  int64_t N = s->N, nl = s->nl;
  int m = s->p.m;
  free_y(s);
  s->ycnt = xcalloc((size_t)nl, sizeof(int64_t));
  s->ynode = xcalloc((size_t)nl, sizeof(int64_t *));
  s->yval = xcalloc((size_t)nl, sizeof(double *));
  double *u = xcalloc((size_t)(N * dim), sizeof(double));
  double *v = xcalloc((size_t)(N * dim), sizeof(double));
  double *a = xcalloc((size_t)(N * dim), sizeof(double));
  double *f = xcalloc((size_t)(N * dim), sizeof(double));
  int64_t *ball = xcalloc((size_t)N, sizeof(int64_t));
  int64_t *slot = xcalloc((size_t)N, sizeof(int64_t));
  if (!s->ycnt || !s->ynode || !s->yval || !u || !v || !a || !f || !ball || !slot) {
    free(u); free(v); free(a); free(f); free(ball); free(slot);
    return -1;
  }
  for (int64_t i = 0; i < N; i++) slot[i] = -1;
  memcpy(s->musnap, s->mu, (size_t)s->nnz); /* Y is built on the current bond states */
  memset(s->H, 0, sizeof(double) * (size_t)(nl * nl));
  double Rr = (double)(m - 1) * s->delta;
  double Rr2 = Rr * Rr;
  for (int64_t c = 0; c < nl; c++) {
    int64_t pnode = s->cn[c / dim];
    int dir = (int)(c % dim);
    int64_t nb = 0;
    for (int64_t i = 0; i < N; i++)
      if (dist2(dim, s->x + pnode * dim, s->x + i * dim) <= Rr2) ball[nb++] = i;
    for (int j = 1; j <= m; j++) {
      double load = (double)j / (double)m;
      for (int64_t b = 0; b < nb; b++) {
        int64_t i = ball[b];
        for (int d = 0; d < dim; d++)
          u[i * dim + d] = (u[i * dim + d] + s->dtP * v[i * dim + d]) + s->hdt2P * a[i * dim + d];
      }
      for (int64_t b = 0; b < nb; b++) {
        int64_t i = ball[b];
        double F[3];
        node_force(s, i, u, s->musnap, 0, F);
        for (int d = 0; d < dim; d++) f[i * dim + d] = F[d];
      }
      for (int64_t b = 0; b < nb; b++) {
        int64_t i = ball[b];
        for (int d = 0; d < dim; d++) {
          double fl = f[i * dim + d];
          if (i == pnode && d == dir) fl = fl + load;
          double an = fl / s->mP[i];
          v[i * dim + d] = v[i * dim + d] + s->hdtP * (a[i * dim + d] + an);
          a[i * dim + d] = an;
        }
      }
    }
    s->ycnt[c] = nb;
    s->ynode[c] = malloc(sizeof(int64_t) * (size_t)(nb ? nb : 1));
    s->yval[c] = malloc(sizeof(double) * (size_t)(nb ? nb : 1) * 3 * dim);
    if (!s->ynode[c] || !s->yval[c]) {
      set_err("out of memory storing Y");
      free(u); free(v); free(a); free(f); free(ball); free(slot);
      return -1;
    }
    for (int64_t b = 0; b < nb; b++) {
      int64_t i = ball[b];
      s->ynode[c][b] = i;
      for (int d = 0; d < dim; d++) {
        s->yval[c][(b * 3 + 0) * dim + d] = u[i * dim + d];
        s->yval[c][(b * 3 + 1) * dim + d] = v[i * dim + d];
        s->yval[c][(b * 3 + 2) * dim + d] = a[i * dim + d];
      }
      slot[i] = b;
    }
    /* H_P column c = G_P Ydot^PD_m e_c */
    for (int64_t q = 0; q < s->nc; q++) {
      int64_t b = slot[s->cn[q]];
      if (b < 0) continue;
      for (int d = 0; d < dim; d++) s->H[(q * dim + d) * nl + c] = s->yval[c][(b * 3 + 1) * dim + d];
    }
    for (int64_t b = 0; b < nb; b++) {
      int64_t i = ball[b];
      slot[i] = -1;
      for (int d = 0; d < dim; d++) u[i * dim + d] = v[i * dim + d] = a[i * dim + d] = 0.0;
    }
  }
  if (s->beta > 0.0) {
    /* + gamma dt_FE G_F A^-1 G_F^T  (-G_F Ydot^FE of the implicit FE step) */
    int64_t nF = s->nfe * dim;
    double *x = xcalloc((size_t)nF, sizeof(double));
    if (!x) { free(u); free(v); free(a); free(f); free(ball); free(slot); return -1; }
    for (int64_t c = 0; c < nl; c++) {
      int64_t qq = c / dim;
      int dc = (int)(c % dim);
      memset(x, 0, sizeof(double) * (size_t)nF);
      for (int aq = 0; aq < s->nen; aq++) {
        int64_t t = (int64_t)s->conn[s->cel[qq] * s->nen + aq] * dim + dc;
        if (fe_free_dof(s, t)) x[t] += s->cw[qq * s->nen + aq];
      }
      fe_solve(s, x, x);
      for (int64_t pq = 0; pq < s->nc; pq++)
        for (int dp = 0; dp < dim; dp++) {
          double g = 0.0;
          for (int ap = 0; ap < s->nen; ap++) {
            int64_t t = (int64_t)s->conn[s->cel[pq] * s->nen + ap] * dim + dp;
            if (fe_free_dof(s, t)) g += s->cw[pq * s->nen + ap] * x[t];
          }
          s->H[(pq * dim + dp) * nl + c] += s->hdtF * g; /* gamma = 1/2 */
        }
    }
    free(x);
  } else
  /* + 1/2 dt_FE G_F M_F^-1 G_F^T  (-G_F Ydot^FE) */
  for (int64_t pq = 0; pq < s->nc; pq++)
    for (int64_t qq = 0; qq < s->nc; qq++) {
      double acc[3] = {0, 0, 0};
      for (int ap = 0; ap < s->nen; ap++)
        for (int aq = 0; aq < s->nen; aq++) {
          int64_t np_ = s->conn[s->cel[pq] * s->nen + ap];
          int64_t nq_ = s->conn[s->cel[qq] * s->nen + aq];
          if (np_ != nq_) continue;
          for (int d = 0; d < dim; d++) {
            if (s->bc[np_ * dim + d]) continue;
            acc[d] += s->cw[pq * s->nen + ap] * s->cw[qq * s->nen + aq] / s->mF[np_];
          }
        }
      for (int d = 0; d < dim; d++) s->H[(pq * dim + d) * nl + qq * dim + d] += s->hdtF * acc[d];
    }
  /* Cholesky H = L L^T */
  memcpy(s->L, s->H, sizeof(double) * (size_t)(nl * nl));
  for (int64_t j = 0; j < nl; j++) {
    double d = s->L[j * nl + j];
    for (int64_t k = 0; k < j; k++) d -= s->L[j * nl + k] * s->L[j * nl + k];
    if (!(d > 0.0)) {
      set_err("multiplier matrix not positive definite at row %lld", (long long)j);
      free(u); free(v); free(a); free(f); free(ball); free(slot);
      return -1;
    }
    double ljj = sqrt(d);
    s->L[j * nl + j] = ljj;
    for (int64_t i = j + 1; i < nl; i++) {
      double t = s->L[i * nl + j];
      for (int64_t k = 0; k < j; k++) t -= s->L[i * nl + k] * s->L[j * nl + k];
      s->L[i * nl + j] = t / ljj;
    }
  }
  free(u); free(v); free(a); free(f); free(ball); free(slot);
  return 0;
}

/* Implicit PD step (Eq. 38 with beta = 1/4 for the PD subdomain, pure-PD
 * mode): A = M + beta dt^2 K_PD assembled column by column from the linear
 * bond force of Eq. 2 with the current bond states (K_PD u = -f(u)), and
 * factored (Cholesky, A = L L^T).  Rebuilt whenever bonds break. */
static int build_pd_implicit(orc_solver *s) {
  int dim = s->dim;
  int64_t n = s->N * dim;
  double c = s->betaP * s->dtP * s->dtP;
  if (!s->LP) s->LP = xcalloc((size_t)(n * n), sizeof(double));
  double *A = s->LP;
  double *e = xcalloc((size_t)n, sizeof(double));
  if (!A || !e) { free(e); return -1; }
  for (int64_t j = 0; j < n; j++) {
    e[j] = 1.0;
    for (int64_t i = 0; i < s->N; i++) {
      double F[3];
      node_force(s, i, e, s->mu, 0, F); /* column j of -K_PD */
      for (int d = 0; d < dim; d++) A[(i * dim + d) * n + j] = -c * F[d];
    }
    e[j] = 0.0;
    A[j * n + j] += s->mP[j / dim];
  }
  free(e);
  for (int64_t j = 0; j < n; j++) {
    double d = A[j * n + j];
    for (int64_t k = 0; k < j; k++) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0)) { set_err("implicit PD matrix not positive definite at row %lld", (long long)j); return -1; }
    double ljj = sqrt(d);
    A[j * n + j] = ljj;
    for (int64_t i = j + 1; i < n; i++) {
      double t = A[i * n + j];
      for (int64_t k = 0; k < j; k++) t -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = t / ljj;
    }
  }
  return 0;
}

/* x = A^-1 b through the implicit PD factor (x and b may alias). */
static void pd_solve(const orc_solver *s, const double *b, double *x) {
  int64_t n = s->N * s->dim;
  const double *L = s->LP;
  for (int64_t i = 0; i < n; i++) {
    double t = b[i];
    for (int64_t k = 0; k < i; k++) t -= L[i * n + k] * x[k];
    x[i] = t / L[i * n + i];
  }
  for (int64_t i = n - 1; i >= 0; i--) {
    double t = x[i];
    for (int64_t k = i + 1; k < n; k++) t -= L[k * n + i] * x[k];
    x[i] = t / L[i * n + i];
  }
}

/* ------------------------------------------------------------------------- */
/* Create                                                                    */
/* ------------------------------------------------------------------------- */
orc_solver *orc_create(const orc_problem *p) {
  if (p->dim != 2 && p->dim != 3) { set_err("dim must be 2 or 3"); return NULL; }
  if (p->mode != ORC_COUPLED && p->mode != ORC_PURE_PD && p->mode != ORC_PURE_FE) { set_err("bad mode"); return NULL; }
  if (p->mode != ORC_PURE_FE && (p->n_pd <= 0 || !p->pos)) { set_err("no PD nodes"); return NULL; }
  if (p->mode == ORC_PURE_PD && (p->traction_x != 0.0 || p->clamp_x0)) {
    set_err("traction_x and clamp_x0 act on the FE mesh");
    return NULL;
  }
  if (p->clamp_x0 && p->vel_bc != 0.0) { set_err("clamp_x0 needs vel_bc = 0"); return NULL; }
  if (p->pd_beta != 0.0 && (p->pd_beta != 0.25 || p->mode != ORC_PURE_PD)) {
    set_err("pd_beta must be 0, or 1/4 in pure-PD mode");
    return NULL;
  }
  if (p->m < 1) { set_err("m must be >= 1"); return NULL; }
  if (!(p->dx > 0.0) || !(p->horizon_factor >= 1.0)) { set_err("bad dx / horizon"); return NULL; }
  if (!(p->dt_pd > 0.0)) { set_err("dt_pd must be > 0"); return NULL; }
  orc_solver *s = xcalloc(1, sizeof(orc_solver));
  if (!s) return NULL;
  s->p = *p;
  int dim = s->dim = p->dim;
  int64_t N = s->N = p->mode == ORC_PURE_FE ? 0 : p->n_pd; /* the FE-only model has no PD nodes */
  s->x = xcalloc((size_t)(N * dim), sizeof(double));
  if (!s->x) { orc_destroy(s); return NULL; }
  if (N) memcpy(s->x, p->pos, sizeof(double) * (size_t)(N * dim));
  s->nu = dim == 2 ? 1.0 / 3.0 : 0.25;
  s->delta = p->horizon_factor * p->dx;
  s->d2 = s->delta * s->delta;
  s->V = dim == 2 ? p->dx * p->dx * p->thickness : p->dx * p->dx * p->dx;
  s->VV = s->V * s->V;
  /* micromodulus calibration (reading R2): 2D h int c r^5 = 3E/pi, 3D int c r^6 = 3E/pi */
  double E = p->E, pi = 3.14159265358979323846, dl = s->delta;
  double I6, I7;
  if (p->kernel == ORC_K_EXP) {
    s->lexp = dl * p->l_over_delta;
    if (dim == 2) s->c0 = 3.0 * E / (pi * p->thickness * orc_exp_moment(5, dl, s->lexp));
    else s->c0 = 3.0 * E / (pi * orc_exp_moment(6, dl, s->lexp));
    I6 = s->c0 * orc_exp_moment(6, dl, s->lexp);
    I7 = s->c0 * orc_exp_moment(7, dl, s->lexp);
  } else {
    if (dim == 2) s->c0 = 9.0 * E / (pi * p->thickness * dl * dl * dl);
    else s->c0 = 12.0 * E / (pi * dl * dl * dl * dl);
    I6 = s->c0 * dl * dl * dl * dl / 4.0;
    I7 = s->c0 * dl * dl * dl * dl * dl / 5.0;
  }
  /* critical stretch from G0 (reading R4): 2D G0 = h s^2 int c r^6, 3D G0 = pi/2 s^2 int c r^7 */
  if (p->s_crit > 0.0) s->scrit = p->s_crit;
  else if (dim == 2) s->scrit = sqrt(p->G0 / (p->thickness * I6));
  else s->scrit = sqrt(2.0 * p->G0 / (pi * I7));
  s->dtP = p->dt_pd;
  s->hdtP = 0.5 * s->dtP;
  s->hdt2P = 0.5 * s->dtP * s->dtP;
  s->dtF = (double)p->m * s->dtP;
  s->hdtF = 0.5 * s->dtF;
  s->hdt2F = 0.5 * s->dtF * s->dtF;
  /* Omega^2: the PD box shrunk by l^O on faces not on the body boundary (R9) */
  for (int a = 0; a < dim; a++) {
    double tol = 1e-9 * (p->dom_hi[a] - p->dom_lo[a]);
    s->o2lo[a] = p->pd_lo[a] + (fabs(p->pd_lo[a] - p->dom_lo[a]) > tol ? p->overlap : 0.0);
    s->o2hi[a] = p->pd_hi[a] - (fabs(p->pd_hi[a] - p->dom_hi[a]) > tol ? p->overlap : 0.0);
  }
  /* neighbour lists */
  int64_t cap = N * 8;
  for (;;) {
    s->rp = xcalloc((size_t)N + 1, sizeof(int64_t));
    s->col = xcalloc((size_t)cap, sizeof(int32_t));
    if (!s->rp || !s->col) { orc_destroy(s); return NULL; }
    int64_t nnz = N <= 4096 ? orc_neighbors_brute(dim, N, s->x, s->delta, s->rp, s->col, cap)
                            : orc_neighbors_grid(dim, N, s->x, s->delta, s->rp, s->col, cap);
    if (nnz >= 0) { s->nnz = nnz; break; }
    free(s->rp); free(s->col); s->rp = NULL; s->col = NULL;
    cap *= 2;
  }
  s->mu = xcalloc((size_t)s->nnz, 1);
  s->musnap = xcalloc((size_t)s->nnz, 1);
  s->alpha = xcalloc((size_t)N, sizeof(double));
  s->mP = xcalloc((size_t)N, sizeof(double));
  s->uP = xcalloc((size_t)(N * dim), sizeof(double));
  s->vP = xcalloc((size_t)(N * dim), sizeof(double));
  s->aP = xcalloc((size_t)(N * dim), sizeof(double));
  s->PP = xcalloc((size_t)(N * dim), sizeof(double));
  s->region = xcalloc((size_t)N, 1);
  if (!s->mu || !s->musnap || !s->alpha || !s->mP || !s->uP || !s->vP || !s->aP || !s->PP ||
      !s->region) { orc_destroy(s); return NULL; }
  for (int64_t i = 0; i < N; i++)
    for (int64_t t = s->rp[i]; t < s->rp[i + 1]; t++) s->mu[t] = crosses_crack(s, i, s->col[t]) ? 0 : 1;
  for (int64_t i = 0; i < N; i++) {
    s->alpha[i] = alpha_at(s, s->x + i * dim);
    if (s->alpha[i] >= 1.0) { set_err("PD node %lld has alpha = 1", (long long)i); orc_destroy(s); return NULL; }
    s->mP[i] = (1.0 - s->alpha[i]) * p->rho * s->V; /* reading R10 */
  }
  if (p->mode == ORC_PURE_PD) {
    /* tractions as a body force T/delta over a layer of width delta (Sec. 3.3, Sec. 4.1) */
    for (int64_t i = 0; i < N; i++) {
      double y = s->x[i * dim + 1];
      if (y - p->pd_lo[1] < s->delta) s->PP[i * dim + 1] = -p->traction / s->delta * s->V;
      else if (p->pd_hi[1] - y < s->delta) s->PP[i * dim + 1] = p->traction / s->delta * s->V;
    }
  } else {
    if (p->fe_n[0] < 1 || p->fe_n[1] < 1 || (dim == 3 && p->fe_n[2] < 1) || !(p->fe_h > 0.0)) {
      set_err("coupled and FE-only modes need an FE mesh");
      orc_destroy(s);
      return NULL;
    }
    if (build_fe(s)) { orc_destroy(s); return NULL; }
    s->beta = p->fe_beta;
    if (s->beta != 0.0 && !(s->beta == 0.25)) { set_err("fe_beta must be 0 or 1/4"); orc_destroy(s); return NULL; }
    if (s->beta > 0.0 && build_fe_implicit(s)) { orc_destroy(s); return NULL; }
    /* constraints at every PD node of the overlap (reading R12) */
    for (int64_t i = 0; i < N; i++) if (s->alpha[i] > 0.0) s->nc++;
    s->nl = s->nc * dim;
    s->cn = xcalloc((size_t)s->nc, sizeof(int64_t));
    s->cidx = xcalloc((size_t)N, sizeof(int64_t));
    if (!s->cidx) { orc_destroy(s); return NULL; }
    for (int64_t i = 0; i < N; i++) s->cidx[i] = -1;
    s->cel = xcalloc((size_t)s->nc, sizeof(int64_t));
    s->cw = xcalloc((size_t)(s->nc * s->nen), sizeof(double));
    const int full = !p->setup_only;
    if (full) {
      s->H = xcalloc((size_t)(s->nl * s->nl), sizeof(double));
      s->L = xcalloc((size_t)(s->nl * s->nl), sizeof(double));
    }
    s->lam0 = xcalloc((size_t)s->nl, sizeof(double));
    if (!s->cn || !s->cel || !s->cw || (full && (!s->H || !s->L)) || !s->lam0) { orc_destroy(s); return NULL; }
    int64_t q = 0;
    double h = p->fe_h;
    for (int64_t i = 0; i < N; i++) {
      if (!(s->alpha[i] > 0.0)) continue;
      s->cn[q] = i;
      s->cidx[i] = q;
      int64_t ei[3] = {0, 0, 0};
      double xi[3] = {0, 0, 0};
      for (int a = 0; a < dim; a++) {
        double t = (s->x[i * dim + a] - p->dom_lo[a]) / h;
        ei[a] = (int64_t)floor(t);
        if (ei[a] >= p->fe_n[a]) ei[a] = p->fe_n[a] - 1;
        if (ei[a] < 0) ei[a] = 0;
        xi[a] = 2.0 * (t - (double)ei[a]) - 1.0;
      }
      int64_t e = (ei[2] * p->fe_n[1] + ei[1]) * p->fe_n[0] + ei[0];
      if (!s->eact[e]) { set_err("constraint node %lld lies in an inactive element", (long long)i); orc_destroy(s); return NULL; }
      s->cel[q] = e;
      for (int a = 0; a < s->nen; a++) s->cw[q * s->nen + a] = shape(dim, a, xi); /* G_F row: N_a(x_p) */
      q++;
    }
    if (full) {
      double Rr = (double)(p->m - 1) * s->delta;
      double Rr2 = Rr * Rr;
      for (int64_t i = 0; i < N; i++)
        for (int64_t c = 0; c < s->nc; c++)
          if (dist2(dim, s->x + s->cn[c] * dim, s->x + i * dim) <= Rr2) {
            s->region[i] = 1;
            s->nregion++;
            break;
          }
      if (build_y(s)) { orc_destroy(s); return NULL; }
    }
  }
  s->betaP = p->pd_beta;
  if (s->betaP > 0.0 && build_pd_implicit(s)) { orc_destroy(s); return NULL; }
  /* initial accelerations a0 = M^-1 (P - K u0) with u0 = 0 (reading R15) */
  for (int64_t i = 0; i < N; i++)
    for (int d = 0; d < dim; d++) s->aP[i * dim + d] = s->PP[i * dim + d] / s->mP[i];
  return s;
}

void orc_destroy(orc_solver *s) {
  if (!s) return;
  free_y(s);
  free(s->x); free(s->rp); free(s->col); free(s->mu); free(s->musnap);
  free(s->alpha); free(s->mP); free(s->uP); free(s->vP); free(s->aP); free(s->PP);
  free(s->conn); free(s->eact); free(s->nact); free(s->bc); free(s->xF); free(s->gpa);
  free(s->mF); free(s->uF); free(s->vF); free(s->aF); free(s->PF);
  free(s->cn); free(s->cidx); free(s->cel); free(s->cw); free(s->H); free(s->L); free(s->lam0);
  free(s->region);
  free(s->LA);
  free(s->LP);
  free(s->febuf);
  free(s);
}

/* ------------------------------------------------------------------------- */
/* One macro step of Algorithm 1, explicit / explicit (gamma = 1/2, beta = 0) */
/* ------------------------------------------------------------------------- */
static int macro_step(orc_solver *s) {
  int dim = s->dim, m = s->p.m;
  int64_t N = s->N;
  /* the FE-only model takes the coupled path with no constraints: the FE free
   * step is then the whole step */
  int coupled = s->p.mode != ORC_PURE_PD;
  int64_t nF = coupled ? s->nfe * dim : 1;
  int region_broke = 0;
  double *fP = xcalloc((size_t)(N * dim), sizeof(double));
  double *ut = xcalloc((size_t)nF, sizeof(double));
  double *vt = xcalloc((size_t)nF, sizeof(double));
  double *at = xcalloc((size_t)nF, sizeof(double));
  double *fF = xcalloc((size_t)nF, sizeof(double));
  double *tF = xcalloc((size_t)nF, sizeof(double));
  double *r = xcalloc((size_t)(coupled ? s->nl : 1), sizeof(double));
  double *lam = xcalloc((size_t)(coupled ? s->nl : 1), sizeof(double));
  double *W = xcalloc((size_t)(coupled ? N * dim * 3 : (s->betaP > 0.0 ? N * dim : 1)), sizeof(double));
  int rc = -1;
  if (!fP || !ut || !vt || !at || !fF || !tF || !r || !lam || !W) goto out;

  if (coupled && s->beta > 0.0) {
    /* FE free problem (Eq. 47a) with the implicit Newmark step (Eq. 38,
     * gamma = 1/2, beta = 1/4): predictors, then A a~ = P - K u* */
    double b2 = (0.5 - s->beta) * s->dtF * s->dtF;
    for (int64_t n = 0; n < s->nfe; n++) {
      if (!s->nact[n]) continue;
      for (int d = 0; d < dim; d++) {
        int64_t t = n * dim + d;
        if (s->bc[t]) ut[t] = s->uF[t] + s->dtF * s->p.vel_bc;
        else ut[t] = (s->uF[t] + s->dtF * s->vF[t]) + b2 * s->aF[t];
      }
    }
    orc_fe_force(s, ut, fF);
    for (int64_t t = 0; t < s->nfe * dim; t++) at[t] = fe_free_dof(s, t) ? s->PF[t] - fF[t] : 0.0;
    fe_solve(s, at, at);
    for (int64_t n = 0; n < s->nfe; n++) {
      if (!s->nact[n]) continue;
      for (int d = 0; d < dim; d++) {
        int64_t t = n * dim + d;
        if (s->bc[t]) {
          at[t] = 0.0;
          vt[t] = s->p.vel_bc;
        } else {
          ut[t] = ut[t] + s->beta * s->dtF * s->dtF * at[t];
          vt[t] = (s->vF[t] + s->hdtF * s->aF[t]) + s->hdtF * at[t];
        }
      }
    }
  } else if (coupled) {
    /* FE free problem (Eq. 47a, Newmark Eq. 38 with beta = 0) over dt_FE */
    for (int64_t n = 0; n < s->nfe; n++) {
      if (!s->nact[n]) continue;
      for (int d = 0; d < dim; d++) {
        int64_t t = n * dim + d;
        if (s->bc[t]) ut[t] = s->uF[t] + s->dtF * s->p.vel_bc;
        else ut[t] = (s->uF[t] + s->dtF * s->vF[t]) + s->hdt2F * s->aF[t];
      }
    }
    orc_fe_force(s, ut, fF);
    for (int64_t n = 0; n < s->nfe; n++) {
      if (!s->nact[n]) continue;
      for (int d = 0; d < dim; d++) {
        int64_t t = n * dim + d;
        if (s->bc[t]) {
          at[t] = 0.0;
          vt[t] = s->p.vel_bc;
        } else {
          at[t] = (s->PF[t] - fF[t]) / s->mF[n];
          vt[t] = s->vF[t] + s->hdtF * (s->aF[t] + at[t]);
        }
      }
    }
  }

  /* PD free problem (Eq. 48a): m substeps at dt_PD, bond states updated on the
   * free problem only (Sec. 2.5, note on broken bonds) */
  for (int j = 1; j <= m; j++) {
    if (s->betaP > 0.0) {
      /* implicit PD step (Eq. 38, beta = 1/4, pure-PD mode): predictor, then
       * (M + beta dt^2 K) a = P + f(u*) with the current bond states; the
       * critical-stretch test runs on the solved displacement and its breaks
       * take effect from the next step (reading R36) */
      double b2 = (0.5 - s->betaP) * s->dtP * s->dtP, c = s->betaP * s->dtP * s->dtP;
      double *us = W; /* N dim scratch (the link buffers are unused in pure-PD mode) */
      for (int64_t t = 0; t < N * dim; t++) us[t] = (s->uP[t] + s->dtP * s->vP[t]) + b2 * s->aP[t];
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < N; i++) {
        double F[3];
        node_force(s, i, us, s->mu, 0, F);
        for (int d = 0; d < dim; d++) fP[i * dim + d] = F[d] + s->PP[i * dim + d];
      }
      pd_solve(s, fP, fP);
      for (int64_t t = 0; t < N * dim; t++) {
        double an = fP[t];
        s->uP[t] = us[t] + c * an;
        s->vP[t] = s->vP[t] + s->hdtP * (s->aP[t] + an);
        s->aP[t] = an;
      }
      int64_t broke_j = 0;
#pragma omp parallel for schedule(static) reduction(+ : broke_j)
      for (int64_t i = 0; i < N; i++) {
        double F[3];
        broke_j += node_force(s, i, s->uP, s->mu, s->p.breaking, F);
      }
      s->nbroken += broke_j;
      if (broke_j && build_pd_implicit(s)) goto out;
      s->pd_steps++;
      continue;
    }
    double sfac = 1.0 - (double)j / (double)m; /* S_j = (1 - j/m) lambda_0 (reading R14) */
    /* The loops over nodes below are independent per node (each node sums its
     * own family and owns its row of bond states), so an OpenMP build gives
     * identical results; without -fopenmp the pragmas are ignored. */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++)
      for (int d = 0; d < dim; d++) {
        int64_t t = i * dim + d;
        s->uP[t] = (s->uP[t] + s->dtP * s->vP[t]) + s->hdt2P * s->aP[t];
      }
    int64_t broke_j = 0;
    int region_j = 0;
#pragma omp parallel for schedule(static) reduction(+ : broke_j) reduction(| : region_j)
    for (int64_t i = 0; i < N; i++) {
      double F[3];
      int64_t b = node_force(s, i, s->uP, s->mu, s->p.breaking, F);
      if (b) {
        broke_j += b;
        if (s->region[i]) region_j = 1;
      }
      for (int d = 0; d < dim; d++) fP[i * dim + d] = F[d];
    }
    s->nbroken += broke_j;
    if (region_j) region_broke = 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
      int64_t q = coupled ? s->cidx[i] : -1;
      for (int d = 0; d < dim; d++) {
        int64_t t = i * dim + d;
        double fl = fP[t] + s->PP[t];
        if (q >= 0) fl = fl + sfac * s->lam0[q * dim + d]; /* + G_P^T S_j */
        double an = fl / s->mP[i];
        s->vP[t] = s->vP[t] + s->hdtP * (s->aP[t] + an);
        s->aP[t] = an;
      }
    }
    s->pd_steps++;
  }

  if (coupled) {
    int64_t nl = s->nl;
    /* right-hand side of Eq. 49: G_F v~_F - G_P V_m (velocity continuity, Eq. 41) */
    for (int64_t q = 0; q < s->nc; q++)
      for (int d = 0; d < dim; d++) {
        double g = 0.0;
        for (int a = 0; a < s->nen; a++)
          g += s->cw[q * s->nen + a] * vt[(int64_t)s->conn[s->cel[q] * s->nen + a] * dim + d];
        r[q * dim + d] = g - s->vP[s->cn[q] * dim + d];
      }
    /* H lambda_m = r through the Cholesky factor */
    for (int64_t i = 0; i < nl; i++) {
      double t = r[i];
      for (int64_t k = 0; k < i; k++) t -= s->L[i * nl + k] * lam[k];
      lam[i] = t / s->L[i * nl + i];
    }
    for (int64_t i = nl - 1; i >= 0; i--) {
      double t = lam[i];
      for (int64_t k = i + 1; k < nl; k++) t -= s->L[k * nl + i] * lam[k];
      lam[i] = t / s->L[i * nl + i];
    }
    /* FE update: U = V + Y^FE lambda, Y^FE = (-M^-1 G_F^T, -dt/2 M^-1 G_F^T, 0) */
    for (int64_t q = 0; q < s->nc; q++)
      for (int a = 0; a < s->nen; a++) {
        int64_t n = s->conn[s->cel[q] * s->nen + a];
        for (int d = 0; d < dim; d++) tF[n * dim + d] += s->cw[q * s->nen + a] * lam[q * dim + d];
      }
    if (s->beta > 0.0) {
      /* implicit FE link response: A dA = -G_F^T lambda; da, gamma dt dA, beta dt^2 dA */
      for (int64_t t = 0; t < s->nfe * dim; t++)
        if (!fe_free_dof(s, t)) tF[t] = 0.0;
      fe_solve(s, tF, tF);
      for (int64_t n = 0; n < s->nfe; n++) {
        if (!s->nact[n]) continue;
        for (int d = 0; d < dim; d++) {
          int64_t t = n * dim + d;
          s->uF[t] = ut[t] - s->beta * s->dtF * s->dtF * tF[t];
          s->vF[t] = vt[t] - s->hdtF * tF[t];
          s->aF[t] = at[t] - tF[t];
        }
      }
    } else
    for (int64_t n = 0; n < s->nfe; n++) {
      if (!s->nact[n]) continue;
      for (int d = 0; d < dim; d++) {
        int64_t t = n * dim + d;
        s->uF[t] = ut[t];
        if (s->bc[t]) {
          s->vF[t] = vt[t];
          s->aF[t] = at[t];
        } else {
          double g = tF[t] / s->mF[n];
          s->aF[t] = at[t] - g;
          s->vF[t] = vt[t] - s->hdtF * g;
        }
      }
    }
    /* PD update: U = V + Y^PD lambda_m */
    for (int64_t c = 0; c < nl; c++) {
      double lc = lam[c];
      for (int64_t b = 0; b < s->ycnt[c]; b++) {
        int64_t i = s->ynode[c][b];
        for (int k = 0; k < 3; k++)
          for (int d = 0; d < dim; d++)
            W[(k * N + i) * dim + d] += s->yval[c][(b * 3 + k) * dim + d] * lc;
      }
    }
    for (int64_t t = 0; t < N * dim; t++) {
      s->uP[t] = s->uP[t] + W[t];
      s->vP[t] = s->vP[t] + W[N * dim + t];
      s->aP[t] = s->aP[t] + W[2 * N * dim + t];
    }
    memcpy(s->lam0, lam, sizeof(double) * (size_t)nl);
    /* rebuild Y^PD when a bond inside its support broke (Alg. 1, last step) */
    if (m >= 2 && region_broke) {
      if (build_y(s)) goto out;
      s->nrebuild++;
    }
  }
  s->macro_steps++;
  rc = 0;
out:
  free(fP); free(ut); free(vt); free(at); free(fF); free(tF); free(r); free(lam); free(W);
  return rc;
}

int orc_advance(orc_solver *s, int64_t n) {
  if (s->p.setup_only) {
    set_err("setup-only oracle instance cannot advance");
    return -1;
  }
  for (int64_t k = 0; k < n; k++)
    if (macro_step(s)) return -1;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Accessors                                                                 */
/* ------------------------------------------------------------------------- */
int orc_constraint_residual(orc_solver *s, double *out) {
  if (s->p.mode != ORC_COUPLED) return -1;
  int dim = s->dim;
  for (int64_t q = 0; q < s->nc; q++)
    for (int d = 0; d < dim; d++) {
      double g = 0.0;
      for (int a = 0; a < s->nen; a++)
        g += s->cw[q * s->nen + a] * s->vF[(int64_t)s->conn[s->cel[q] * s->nen + a] * dim + d];
      out[q * dim + d] = g - s->vP[s->cn[q] * dim + d];
    }
  return 0;
}

int orc_info_get(orc_solver *s, orc_info *o) {
  int dim = s->dim;
  memset(o, 0, sizeof *o);
  o->delta = s->delta; o->volume = s->V; o->c0 = s->c0; o->s_crit = s->scrit; o->nu = s->nu;
  o->dt_pd = s->dtP; o->dt_fe = s->dtF;
  o->n_pd = s->N; o->nnz = s->nnz; o->n_fe_nodes = s->nfe; o->n_fe_elems = s->ne;
  o->n_constraints = s->nc; o->n_region = s->nregion;
  o->pd_steps = s->pd_steps; o->macro_steps = s->macro_steps;
  o->n_rebuilds = s->nrebuild; o->n_broken = s->nbroken;
  double ek = 0.0, w = 0.0;
  for (int64_t i = 0; i < s->N; i++)
    for (int d = 0; d < dim; d++) {
      double v = s->vP[i * dim + d];
      ek += 0.5 * s->mP[i] * v * v;
      w += s->PP[i * dim + d] * s->uP[i * dim + d];
    }
  o->e_pd = orc_pd_energy(s, s->uP);
  if (s->p.mode != ORC_PURE_PD) {
    double *f = xcalloc((size_t)(s->nfe * dim), sizeof(double));
    if (!f) return -1;
    orc_fe_force(s, s->uF, f);
    double ef = 0.0;
    for (int64_t n = 0; n < s->nfe; n++) {
      if (!s->nact[n]) continue;
      for (int d = 0; d < dim; d++) {
        double v = s->vF[n * dim + d];
        ek += 0.5 * s->mF[n] * v * v;
        w += s->PF[n * dim + d] * s->uF[n * dim + d];
        ef += 0.5 * s->uF[n * dim + d] * f[n * dim + d];
      }
    }
    free(f);
    o->e_fe = ef;
  }
  o->e_kin = ek;
  o->w_ext = w;
  return 0;
}

int64_t orc_get(orc_solver *s, int what, double *out, int64_t cap) {
  int dim = s->dim;
  int64_t n = 0;
  const double *src = NULL;
  switch (what) {
    case ORC_PD_U: src = s->uP; n = s->N * dim; break;
    case ORC_PD_V: src = s->vP; n = s->N * dim; break;
    case ORC_PD_A: src = s->aP; n = s->N * dim; break;
    case ORC_PD_ALPHA: src = s->alpha; n = s->N; break;
    case ORC_PD_MASS: src = s->mP; n = s->N; break;
    case ORC_PD_P: src = s->PP; n = s->N * dim; break;
    case ORC_FE_U: src = s->uF; n = s->nfe * dim; break;
    case ORC_FE_V: src = s->vF; n = s->nfe * dim; break;
    case ORC_FE_A: src = s->aF; n = s->nfe * dim; break;
    case ORC_FE_MASS: src = s->mF; n = s->nfe; break;
    case ORC_FE_X: src = s->xF; n = s->nfe * dim; break;
    case ORC_FE_P: src = s->PF; n = s->nfe * dim; break;
    case ORC_LAMBDA: src = s->lam0; n = s->nl; break;
    case ORC_H: src = s->H; n = s->nl * s->nl; break;
    case ORC_GF: src = s->cw; n = s->nc * s->nen; break;
    case ORC_DAMAGE:
      n = s->N;
      if (cap < n) return -1;
      for (int64_t i = 0; i < s->N; i++) {
        int64_t fam = s->rp[i + 1] - s->rp[i], in = 0;
        for (int64_t t = s->rp[i]; t < s->rp[i + 1]; t++) in += s->mu[t];
        out[i] = fam > 0 ? 1.0 - (double)in / (double)fam : 0.0; /* Eq. 5, uniform volumes */
      }
      return n;
    case ORC_CONSTRAINT_NODES:
      n = s->nc;
      if (cap < n) return -1;
      for (int64_t q = 0; q < n; q++) out[q] = (double)s->cn[q];
      return n;
    case ORC_GF_NODES:
      n = s->nc * s->nen;
      if (cap < n) return -1;
      for (int64_t q = 0; q < s->nc; q++)
        for (int a = 0; a < s->nen; a++) out[q * s->nen + a] = (double)s->conn[s->cel[q] * s->nen + a];
      return n;
    case ORC_REGION:
      n = s->N;
      if (cap < n) return -1;
      for (int64_t i = 0; i < n; i++) out[i] = (double)s->region[i];
      return n;
    default: return -1;
  }
  if (cap < n) return -1;
  if (n) memcpy(out, src, sizeof(double) * (size_t)n);
  return n;
}

int orc_set(orc_solver *s, int what, const double *in, int64_t n) {
  int dim = s->dim;
  double *dst = NULL;
  int64_t want = 0;
  switch (what) {
    case ORC_PD_U: dst = s->uP; want = s->N * dim; break;
    case ORC_PD_V: dst = s->vP; want = s->N * dim; break;
    case ORC_PD_A: dst = s->aP; want = s->N * dim; break;
    case ORC_FE_U: dst = s->uF; want = s->nfe * dim; break;
    case ORC_FE_V: dst = s->vF; want = s->nfe * dim; break;
    case ORC_FE_A: dst = s->aF; want = s->nfe * dim; break;
    case ORC_LAMBDA: dst = s->lam0; want = s->nl; break;
    default: return -1;
  }
  if (n != want) return -1;
  if (n) memcpy(dst, in, sizeof(double) * (size_t)n);
  return 0;
}

int64_t orc_get_bonds(orc_solver *s, int64_t *row_ptr, int32_t *col, uint8_t *mu, int64_t cap) {
  if (cap < s->nnz) return -1;
  if (row_ptr) memcpy(row_ptr, s->rp, sizeof(int64_t) * (size_t)(s->N + 1));
  if (col) memcpy(col, s->col, sizeof(int32_t) * (size_t)s->nnz);
  if (mu) memcpy(mu, s->mu, (size_t)s->nnz);
  return s->nnz;
}

/* Stable step bounds for velocity Verlet (dt < 2 / omega_max, Sec. 2.4).
 * which = 0: PD, per node sqrt(2 m_i / sum_k w c |xi|^2 V_i V_k).
 * which = 1: FE, power iteration for the largest eigenvalue of M^-1 K.
 * which = 2: FE, Gershgorin bound from element matrices (never optimistic). */
double orc_dt_bound(orc_solver *s, int which) {
  int dim = s->dim;
  if (which == 0) {
    double best = INFINITY;
    for (int64_t i = 0; i < s->N; i++) {
      double k = 0.0;
      for (int64_t t = s->rp[i]; t < s->rp[i + 1]; t++) {
        int64_t j = s->col[t];
        double r2 = dist2(dim, s->x + i * dim, s->x + j * dim);
        double w = 1.0 - 0.5 * (s->alpha[i] + s->alpha[j]);
        k += w * cfun(s, sqrt(r2)) * r2 * s->VV;
      }
      if (k > 0.0) {
        double dt = sqrt(2.0 * s->mP[i] / k);
        if (dt < best) best = dt;
      }
    }
    return best;
  }
  if (s->p.mode == ORC_PURE_PD) return INFINITY;
  int64_t n = s->nfe * dim;
  if (which == 2) {
    double *rowsum = xcalloc((size_t)n, sizeof(double));
    double ue[24], fe[24], eps[6], sig[6], ke[24][24];
    int nd = s->nen * dim;
    for (int64_t e = 0; e < s->ne; e++) {
      if (!s->eact[e]) continue;
      for (int c = 0; c < nd; c++) {
        for (int t = 0; t < nd; t++) ue[t] = (t == c) ? 1.0 : 0.0;
        for (int t = 0; t < nd; t++) fe[t] = 0.0;
        for (int g = 0; g < s->ngp; g++) {
          double al = s->gpa[e * s->ngp + g];
          strain(s, g, ue, eps);
          for (int rr = 0; rr < s->nstr; rr++) {
            sig[rr] = 0.0;
            for (int cc = 0; cc < s->nstr; cc++) sig[rr] += s->D[rr][cc] * eps[cc];
          }
          btsig(s, g, sig, al * s->detJ * s->p.thickness, fe);
        }
        for (int t = 0; t < nd; t++) ke[t][c] = fe[t];
      }
      for (int a = 0; a < nd; a++)
        for (int b = 0; b < nd; b++) {
          int64_t na = s->conn[e * s->nen + a / dim], nb = s->conn[e * s->nen + b / dim];
          rowsum[na * dim + a % dim] += fabs(ke[a][b]) / sqrt(s->mF[na] * s->mF[nb]);
        }
    }
    double lmax = 0.0;
    for (int64_t t = 0; t < n; t++)
      if (!s->bc[t] && rowsum[t] > lmax) lmax = rowsum[t];
    free(rowsum);
    return 2.0 / sqrt(lmax);
  }
  double *xv = xcalloc((size_t)n, sizeof(double)), *f = xcalloc((size_t)n, sizeof(double));
  if (!xv || !f) { free(xv); free(f); return -1.0; }
  uint64_t st = 0x1234567ULL;
  for (int64_t t = 0; t < n; t++) {
    st = st * 6364136223846793005ULL + 1442695040888963407ULL;
    xv[t] = s->nact[t / dim] && !s->bc[t] ? (double)(st >> 11) / 9007199254740992.0 - 0.5 : 0.0;
  }
  double lam = 0.0;
  for (int it = 0; it < 3000; it++) {
    orc_fe_force(s, xv, f);
    double num = 0.0, den = 0.0, nrm = 0.0;
    for (int64_t t = 0; t < n; t++) {
      if (!s->nact[t / dim] || s->bc[t]) { f[t] = 0.0; continue; }
      num += xv[t] * f[t];
      den += xv[t] * xv[t] * s->mF[t / dim];
      f[t] = f[t] / s->mF[t / dim];
      nrm += f[t] * f[t];
    }
    lam = num / den;
    nrm = sqrt(nrm);
    for (int64_t t = 0; t < n; t++) xv[t] = f[t] / nrm;
  }
  free(xv); free(f);
  return 2.0 / sqrt(lam);
}
