/*
 * FP64 CPU oracle for the batched gradient of forward dynamics.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the parity reference for the HIP path.
 * Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * load it; the product library never links, calls or includes anything here, and
 * this directory includes nothing from the product.
 *
 * It is written for a reader checking it against the paper by eye: dense 6x6
 * spatial matrices, plain loops, no blocking or fusion.
 *
 * Conventions (paper Sec. III-B and Eq. 2):
 *   - bodies i = 0..n-1, parent[i] < i, parent -1 = fixed base;
 *   - spatial vectors ordered [angular; linear];
 *   - X_i = X_J(q_i) X_T,i with X_T the fixed parent-to-joint transform given by rotation
 *     E_T and origin r, and X_J the joint's own motion along its axis a_i (a unit vector in
 *     joint coordinates, +z unless given): the rotation by q_i about a_i for a revolute
 *     joint, the translation by q_i a_i for a prismatic one (Sec. IV: joint types);
 *   - S_i = (a_i, 0) for a revolute joint, (0, a_i) for a prismatic joint;
 *   - gravity enters as the fictitious base acceleration a_0 = -g;
 *   - matrices are row-major; dtau_dq[i*n+j] = d tau_i / d q_j.
 */
#ifndef GRID_ORACLE_H
#define GRID_ORACLE_H

#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int n;
    const int *parent;     /* [n] */
    const double *E_T;     /* [n][9] rotation from parent frame to joint frame, row-major */
    const double *r;       /* [n][3] joint origin, parent coordinates */
    const double *mass;    /* [n] */
    const double *com;     /* [n][3] centre of mass, body coordinates */
    const double *Ic;      /* [n][6] xx yy zz xy xz yz, about the centre of mass */
    double gravity[3];     /* base-frame gravity vector */
    const double *axis;    /* [n][3] joint axes in joint coordinates (normalised here);
                              NULL: +z for every joint */
    const int *prismatic;  /* [n] nonzero: prismatic joint, zero: revolute;
                              NULL: every joint revolute */
} orc_model;

/* status: 0 ok, -1 invalid model, -2 matrix not positive definite */

/* Eq. 2: motion cross-product matrix v x and force cross-product v x* = -(v x)^T */
void orc_crm(const double v[6], double out[36]);
void orc_crf(const double v[6], double out[36]);

/* X_i(q) as a dense 6x6 matrix and the spatial inertia I_i */
int orc_joint_transform(const orc_model *m, int i, double q, double X[36]);
int orc_spatial_inertia(const orc_model *m, int i, double Ib[36]);

/* RNEA: tau = ID(q, qd, qdd); optional per-body v, a, f (f accumulated) [n][6] */
int orc_rnea(const orc_model *m, const double *q, const double *qd, const double *qdd,
             int gravity_on, double *tau, double *v, double *a, double *f);

/* CRBA mass matrix M(q) [n][n] */
int orc_crba(const orc_model *m, const double *q, double *M);

/* Minv by Cholesky (primary) and by the direct articulated-body recursion (cross-check) */
int orc_minv_cholesky(const orc_model *m, const double *q, double *Minv);
int orc_minv_direct(const orc_model *m, const double *q, double *Minv);

/* forward dynamics qdd = M^-1 (tau - c(q, qd)) by Cholesky solve */
int orc_fd(const orc_model *m, const double *q, const double *qd, const double *tau,
           double *qdd);

/* analytic gradient of inverse dynamics at (q, qd, qdd) */
int orc_rnea_grad(const orc_model *m, const double *q, const double *qd, const double *qdd,
                  double *dtau_dq, double *dtau_dqd);

/* one knot of the full path: qdd, Minv, dqdd/dq, dqdd/dqd */
int orc_fd_grad(const orc_model *m, const double *q, const double *qd, const double *tau,
                double *qdd, double *Minv, double *dqdd_dq, double *dqdd_dqd);

/* N knots, knot-major arrays; OpenMP over knots. Returns the first failing status. */
int orc_fd_grad_batch(const orc_model *m, int N, const double *q, const double *qd,
                      const double *tau, double *qdd, double *Minv, double *dqdd_dq,
                      double *dqdd_dqd);
int orc_num_threads(void);
void orc_set_num_threads(int k);

/* complex-step instantiations (same source, scalar type double complex) */
int orc_rnea_z(const orc_model *m, const double complex *q, const double complex *qd,
               const double complex *qdd, int gravity_on, double complex *tau);
int orc_fd_z(const orc_model *m, const double complex *q, const double complex *qd,
             const double complex *tau, double complex *qdd);

#ifdef __cplusplus
}
#endif
#endif
