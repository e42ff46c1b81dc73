/*
 * Reference oracle for the multi-time-step (MTS) coupling of bond-based
 * peridynamics (PD) and finite elements (FE) in the Arlequin framework
 * (Zhong, Han, Du, Guo, arXiv 2403.03605).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation
 * that the GPU library is checked against.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code with the HIP library.
 */
#ifndef MTS_ORACLE_H
#define MTS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_COUPLED = 0, ORC_PURE_PD = 1,
       ORC_PURE_FE = 2 /* the FE mesh alone with alpha = 1 (the undecomposed FE model of Sec. 3.2) */ };
enum { ORC_W_CUBIC = 0, ORC_W_LINEAR = 1, ORC_W_CONSTANT = 2 };
enum { ORC_K_PMB = 0, ORC_K_EXP = 1 };

typedef struct {
  int32_t dim, mode, breaking, weight_kind, kernel, m;
  int32_t n_cracks;
  int32_t fe_n[3];
  int64_t n_pd;
  const double *pos;          /* n_pd * dim, node-major */
  double dx, horizon_factor;
  double pd_lo[3], pd_hi[3], dom_lo[3], dom_hi[3];
  double fe_h, overlap;
  double cracks[8][3];        /* horizontal segments: y, x_start, x_end */
  double E, rho, G0, thickness, s_crit, l_over_delta;
  double traction, vel_bc, dt_pd;
  int32_t setup_only;         /* 1: weights, masses, FE mesh and constraint set only
                                 (no link region, no unit-load responses, no stepping);
                                 for checks of large runs against the constraint set */
  double fe_beta;             /* Newmark beta of the FE step: 0 explicit, 1/4 average
                                 acceleration (implicit, gamma = 1/2 in both) */
  double traction_x;          /* uniform traction (+x) on the FE face x = dom_hi: the end
                                 load of the beam of Sec. 3.2 */
  int32_t clamp_x0;           /* 1: every component of the FE nodes on x = dom_lo held at
                                 zero (the beam's fixed end); needs vel_bc = 0 */
  double pd_beta;             /* Newmark beta of the PD step (pure-PD mode): 0 explicit
                                 (velocity Verlet), 1/4 average acceleration (implicit) */
} orc_problem;

typedef struct {
  double delta, volume, c0, s_crit, nu, dt_pd, dt_fe;
  int64_t n_pd, nnz, n_fe_nodes, n_fe_elems, n_constraints, n_region;
  int64_t pd_steps, macro_steps, n_rebuilds, n_broken;
  double e_kin, e_pd, e_fe, w_ext;
} orc_info;

enum {
  ORC_PD_U = 0, ORC_PD_V, ORC_PD_A, ORC_FE_U, ORC_FE_V, ORC_FE_A, ORC_DAMAGE,
  ORC_LAMBDA, ORC_PD_ALPHA, ORC_PD_MASS, ORC_FE_MASS, ORC_FE_X, ORC_H,
  ORC_CONSTRAINT_NODES, ORC_FE_P, ORC_PD_P, ORC_GF, ORC_REGION, ORC_GF_NODES
};

typedef struct orc_solver orc_solver;

const char *orc_last_error(void);

/* Neighbour sets H_i = {k != i : |x_k - x_i|^2 <= delta^2}, rows ascending.
 * Return nnz, or -1 if cap is too small. */
int64_t orc_neighbors_brute(int dim, int64_t n, const double *x, double delta,
                            int64_t *row_ptr, int32_t *col, int64_t cap);
int64_t orc_neighbors_grid(int dim, int64_t n, const double *x, double delta,
                           int64_t *row_ptr, int32_t *col, int64_t cap);

/* Closed form of int_0^delta r^n exp(-r/l) dr. */
double orc_exp_moment(int n, double delta, double l);

orc_solver *orc_create(const orc_problem *p);
void orc_destroy(orc_solver *s);
int orc_advance(orc_solver *s, int64_t n_macro);
int orc_info_get(orc_solver *s, orc_info *out);
int64_t orc_get(orc_solver *s, int what, double *out, int64_t cap);
int orc_set(orc_solver *s, int what, const double *in, int64_t n);
int64_t orc_get_bonds(orc_solver *s, int64_t *row_ptr, int32_t *col, uint8_t *mu, int64_t cap);

/* Internal PD force (no breaking, current bond states) for a displacement field. */
int orc_pd_force(orc_solver *s, const double *u, double *f);
/* PD deformation energy 1/4 sum w c (xi.eta)^2 V V for a displacement field. */
double orc_pd_energy(orc_solver *s, const double *u);
/* FE internal force K_F u (Arlequin-weighted). */
int orc_fe_force(orc_solver *s, const double *u, double *f);
/* G_F v_F - G_P v_P for the current state. */
int orc_constraint_residual(orc_solver *s, double *out);
/* Stable step bounds: which = 0 PD (per-node), 1 FE (power iteration on M^-1 K). */
double orc_dt_bound(orc_solver *s, int which);

#ifdef __cplusplus
}
#endif
#endif
