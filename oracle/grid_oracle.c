/*
 * FP64 CPU oracle for the batched gradient of forward dynamics.
 *
 * TEST INFRASTRUCTURE ONLY: the parity reference for the HIP path (see
 * grid_oracle.h). It follows the paper's problem statement:
 *   - forward dynamics qdd = M^-1 (tau - RNEA(q, qd, 0)) (Sec. IV-B, with the sign
 *     fixed by Eq. 1: M qdd + c = tau);
 *   - the gradient of inverse dynamics, Algorithm 1 (forward pass) followed by its
 *     backward pass (force accumulation towards the root, Sec. IV-C);
 *   - dqdd/du = -M^-1 dRNEA(q, qd, qdd)/du for u in {q, qd} (Sec. IV-B), evaluated
 *     at qdd = FD(q, qd, tau); dqdd/dtau = M^-1.
 * M comes from the composite rigid body algorithm and is inverted by Cholesky; the
 * direct articulated-body inverse (Sec. IV-B) is a second route for the tests.
 */
#include <complex.h>
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "grid_oracle.h"

#define R double
#define FN(x) x##_d
#include "rbd_generic.inc"
#undef R
#undef FN

#define R double complex
#define FN(x) x##_z
#include "rbd_generic.inc"
#undef R
#undef FN

static int check_model(const orc_model *m)
{
    if (!m || m->n <= 0 || !m->parent || !m->E_T || !m->r || !m->mass || !m->com || !m->Ic)
        return -1;
    for (int i = 0; i < m->n; ++i) {
        if (m->parent[i] < -1 || m->parent[i] >= i)
            return -1;
        if (m->axis) {
            const double *a = m->axis + 3 * i;
            const double nrm = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
            if (!(fabs(nrm - 1.0) < 1e-6))
                return -1;
        }
        if (m->prismatic && m->prismatic[i] != 0 && m->prismatic[i] != 1)
            return -1;
    }
    return 0;
}

void orc_crm(const double v[6], double out[36]) { crm_d(v, out); }
void orc_crf(const double v[6], double out[36]) { crf_d(v, out); }

int orc_joint_transform(const orc_model *m, int i, double q, double X[36])
{
    if (check_model(m) || i < 0 || i >= m->n)
        return -1;
    xform_d(m, i, q, X);
    return 0;
}

int orc_spatial_inertia(const orc_model *m, int i, double Ib[36])
{
    if (check_model(m) || i < 0 || i >= m->n)
        return -1;
    inertia_d(m, i, Ib);
    return 0;
}

int orc_rnea(const orc_model *m, const double *q, const double *qd, const double *qdd,
             int gravity_on, double *tau, double *v, double *a, double *f)
{
    if (check_model(m))
        return -1;
    return rnea_d(m, q, qd, qdd, gravity_on, tau, v, a, f);
}

int orc_crba(const orc_model *m, const double *q, double *M)
{
    if (check_model(m))
        return -1;
    return crba_d(m, q, M);
}

int orc_fd(const orc_model *m, const double *q, const double *qd, const double *tau,
           double *qdd)
{
    if (check_model(m))
        return -1;
    return fd_d(m, q, qd, tau, qdd);
}

int orc_rnea_z(const orc_model *m, const double complex *q, const double complex *qd,
               const double complex *qdd, int gravity_on, double complex *tau)
{
    if (check_model(m))
        return -1;
    return rnea_z(m, q, qd, qdd, gravity_on, tau, NULL, NULL, NULL);
}

int orc_fd_z(const orc_model *m, const double complex *q, const double complex *qd,
             const double complex *tau, double complex *qdd)
{
    if (check_model(m))
        return -1;
    return fd_z(m, q, qd, tau, qdd);
}

/* M^-1 column by column from the Cholesky factor */
static int minv_from_M(int n, const double *M, double *Minv)
{
    double *L = malloc(sizeof(double) * n * n);
    double *e = calloc(n, sizeof(double));
    double *x = malloc(sizeof(double) * n);
    int st = (L && e && x) ? cholesky_d(n, M, L) : -1;
    for (int k = 0; !st && k < n; ++k) {
        e[k] = 1;
        chol_solve_d(n, L, e, x);
        e[k] = 0;
        for (int i = 0; i < n; ++i)
            Minv[i * n + k] = x[i];
    }
    free(L); free(e); free(x);
    return st;
}

int orc_minv_cholesky(const orc_model *m, const double *q, double *Minv)
{
    if (check_model(m))
        return -1;
    const int n = m->n;
    double *M = malloc(sizeof(double) * n * n);
    if (!M)
        return -1;
    int st = crba_d(m, q, M);
    if (!st)
        st = minv_from_M(n, M, Minv);
    free(M);
    return st;
}

/*
 * Direct M^-1 (Sec. IV-B): the articulated-body recursion with qd = 0, g = 0 and the
 * identity as n right-hand sides. F_i and P_i are 6 x n; row_i is 1 x n.
 *   inward:  U_i = IA_i S_i, D_i = S_i^T U_i, row_i = (e_i^T - S_i^T F_i) / D_i,
 *            IA_lambda += X^T (IA_i - U_i U_i^T / D_i) X,
 *            F_lambda  += X^T (F_i + U_i row_i)
 *   outward: A = X_i P_lambda (0 at the base), row_i -= U_i^T A / D_i,
 *            P_i = A + S_i row_i;   M^-1[i, :] = row_i
 */
int orc_minv_direct(const orc_model *m, const double *q, double *Minv)
{
    if (check_model(m))
        return -1;
    const int n = m->n;
    double (*X)[36] = malloc(sizeof(double[36]) * n);
    double (*IA)[36] = malloc(sizeof(double[36]) * n);
    double (*U)[6] = malloc(sizeof(double[6]) * n);
    double *D = malloc(sizeof(double) * n);
    double *F = calloc((size_t)n * 6 * n, sizeof(double));  /* F[i][k][col] */
    double *P = calloc((size_t)n * 6 * n, sizeof(double));
    double *row = calloc((size_t)n * n, sizeof(double));
    int st = (X && IA && U && D && F && P && row) ? 0 : -1;
    for (int i = 0; !st && i < n; ++i) {
        xform_d(m, i, q[i], X[i]);
        inertia_d(m, i, IA[i]);
    }
    for (int i = n - 1; !st && i >= 0; --i) {
        const int p = m->parent[i];
        double *Fi = F + (size_t)i * 6 * n;
        double S[6];
        joint_S_d(m, i, S);
        mv6_d(IA[i], S, U[i]);
        D[i] = 0;
        for (int k = 0; k < 6; ++k)
            D[i] += S[k] * U[i][k];
        if (!(D[i] > 0)) {
            st = -2;
            break;
        }
        for (int c = 0; c < n; ++c) {
            double sf = 0;
            for (int k = 0; k < 6; ++k)
                sf += S[k] * Fi[k * n + c];
            row[i * n + c] = ((c == i ? 1.0 : 0.0) - sf) / D[i];
        }
        if (p >= 0) {
            double Ia[36], t[36], u[36];
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b)
                    Ia[a * 6 + b] = IA[i][a * 6 + b] - U[i][a] * U[i][b] / D[i];
            mm6_d(Ia, X[i], t);
            mtm6_d(X[i], t, u);
            for (int k = 0; k < 36; ++k)
                IA[p][k] += u[k];
            double *Fp = F + (size_t)p * 6 * n;
            for (int c = 0; c < n; ++c) {
                double col[6], xc[6];
                for (int k = 0; k < 6; ++k)
                    col[k] = Fi[k * n + c] + U[i][k] * row[i * n + c];
                mtv6_d(X[i], col, xc);
                for (int k = 0; k < 6; ++k)
                    Fp[k * n + c] += xc[k];
            }
        }
    }
    for (int i = 0; !st && i < n; ++i) {
        const int p = m->parent[i];
        double *Pi = P + (size_t)i * 6 * n;
        double S[6];
        joint_S_d(m, i, S);
        for (int c = 0; c < n; ++c) {
            double A[6] = {0, 0, 0, 0, 0, 0};
            if (p >= 0) {
                const double *Pp = P + (size_t)p * 6 * n;
                double col[6];
                for (int k = 0; k < 6; ++k)
                    col[k] = Pp[k * n + c];
                mv6_d(X[i], col, A);
            }
            double UA = 0;
            for (int k = 0; k < 6; ++k)
                UA += U[i][k] * A[k];
            row[i * n + c] -= UA / D[i];
            for (int k = 0; k < 6; ++k)
                Pi[k * n + c] = A[k] + S[k] * row[i * n + c];
        }
    }
    if (!st)
        memcpy(Minv, row, sizeof(double) * n * n);
    free(X); free(IA); free(U); free(D); free(F); free(P); free(row);
    return st;
}

/*
 * Gradient of inverse dynamics at (q, qd, qdd) (Algorithm 1 and its backward pass).
 * For u in {q, qd} and each column j, with dv_0 = da_0 = 0:
 *   outward: dv_i = X_i dv_lambda + [i==j] {(X_i v_lambda) x S_i  if u = q;  S_i  if u = qd}
 *            da_i = X_i da_lambda + (dv_i x) S_i qd_i
 *                   + [i==j] {(X_i a_lambda) x S_i  if u = q;  (v_i x) S_i  if u = qd}
 *            df_i = I_i da_i + (dv_i x*) I_i v_i + (v_i x*) I_i dv_i
 *   inward:  dtau_i/du_j = S_i^T df_i
 *            df_lambda += X_i^T df_i + [i==j and u = q] X_i^T (S_i x*) f_i
 * v, a and the accumulated forces f come from RNEA(q, qd, qdd). The velocity term in
 * da_i uses dv_i (the derivative of v_i, which multiplies S qd_i in the RNEA), and the
 * bracketed source terms act only in the joint's own column.
 */
int orc_rnea_grad(const orc_model *m, const double *q, const double *qd, const double *qdd,
                  double *dtau_dq, double *dtau_dqd)
{
    if (check_model(m))
        return -1;
    const int n = m->n;
    double (*X)[36] = malloc(sizeof(double[36]) * n);
    double (*Ib)[36] = malloc(sizeof(double[36]) * n);
    double (*v)[6] = malloc(sizeof(double[6]) * n);
    double (*a)[6] = malloc(sizeof(double[6]) * n);
    double (*f)[6] = malloc(sizeof(double[6]) * n);
    double (*dv)[6] = malloc(sizeof(double[6]) * n);
    double (*da)[6] = malloc(sizeof(double[6]) * n);
    double (*df)[6] = malloc(sizeof(double[6]) * n);
    double *tau = malloc(sizeof(double) * n);
    int st = (X && Ib && v && a && f && dv && da && df && tau) ? 0 : -1;
    if (!st)
        st = rnea_d(m, q, qd, qdd, 1, tau, &v[0][0], &a[0][0], &f[0][0]);
    double (*S)[6] = malloc(sizeof(double[6]) * n);       /* S_i per joint */
    if (!S)
        st = -1;
    for (int i = 0; !st && i < n; ++i)
        joint_S_d(m, i, S[i]);
    double a0[6] = {0, 0, 0, -m->gravity[0], -m->gravity[1], -m->gravity[2]};
    double zero6[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; !st && i < n; ++i) {
        xform_d(m, i, q[i], X[i]);
        inertia_d(m, i, Ib[i]);
    }
    for (int u = 0; !st && u < 2; ++u) {           /* u = 0: q, u = 1: qd */
        double *out = u == 0 ? dtau_dq : dtau_dqd;
        for (int j = 0; j < n; ++j) {
            for (int i = 0; i < n; ++i) {
                const int p = m->parent[i];
                const double *dvp = p < 0 ? zero6 : dv[p];
                const double *dap = p < 0 ? zero6 : da[p];
                const double *vp = p < 0 ? zero6 : v[p];
                const double *ap = p < 0 ? a0 : a[p];
                double t[6], s[6], w[6];
                mv6_d(X[i], dvp, dv[i]);
                if (i == j) {
                    if (u == 0) {
                        mv6_d(X[i], vp, t);
                        crm_apply_d(t, S[i], s);
                    } else {
                        memcpy(s, S[i], sizeof s);
                    }
                    for (int k = 0; k < 6; ++k)
                        dv[i][k] += s[k];
                }
                mv6_d(X[i], dap, da[i]);
                crm_apply_d(dv[i], S[i], s);
                for (int k = 0; k < 6; ++k)
                    da[i][k] += s[k] * qd[i];
                if (i == j) {
                    if (u == 0) {
                        mv6_d(X[i], ap, t);
                        crm_apply_d(t, S[i], s);
                    } else {
                        crm_apply_d(v[i], S[i], s);
                    }
                    for (int k = 0; k < 6; ++k)
                        da[i][k] += s[k];
                }
                double Iv[6], Idv[6];
                mv6_d(Ib[i], da[i], df[i]);
                mv6_d(Ib[i], v[i], Iv);
                crf_apply_d(dv[i], Iv, w);
                for (int k = 0; k < 6; ++k)
                    df[i][k] += w[k];
                mv6_d(Ib[i], dv[i], Idv);
                crf_apply_d(v[i], Idv, w);
                for (int k = 0; k < 6; ++k)
                    df[i][k] += w[k];
            }
            for (int i = n - 1; i >= 0; --i) {
                const int p = m->parent[i];
                double st_ = 0;
                for (int k = 0; k < 6; ++k)
                    st_ += S[i][k] * df[i][k];
                out[i * n + j] = st_;
                if (p >= 0) {
                    double t[6], s[6];
                    mtv6_d(X[i], df[i], t);
                    for (int k = 0; k < 6; ++k)
                        df[p][k] += t[k];
                    if (u == 0 && i == j) {
                        crf_apply_d(S[i], f[i], s);
                        mtv6_d(X[i], s, t);
                        for (int k = 0; k < 6; ++k)
                            df[p][k] += t[k];
                    }
                }
            }
        }
    }
    free(X); free(Ib); free(v); free(a); free(f); free(dv); free(da); free(df); free(tau);
    free(S);
    return st;
}

int orc_fd_grad(const orc_model *m, const double *q, const double *qd, const double *tau,
                double *qdd, double *Minv, double *dqdd_dq, double *dqdd_dqd)
{
    if (check_model(m))
        return -1;
    const int n = m->n;
    double *M = malloc(sizeof(double) * n * n);
    double *L = malloc(sizeof(double) * n * n);
    double *c = malloc(sizeof(double) * n);
    double *zero = calloc(n, sizeof(double));
    double *b = malloc(sizeof(double) * n);
    double *dq = malloc(sizeof(double) * n * n);
    double *dqd = malloc(sizeof(double) * n * n);
    int st = (M && L && c && zero && b && dq && dqd) ? 0 : -1;
    if (!st)
        st = rnea_d(m, q, qd, zero, 1, c, NULL, NULL, NULL);        /* c = RNEA(q, qd, 0) */
    if (!st)
        st = crba_d(m, q, M);
    if (!st)
        st = cholesky_d(n, M, L);
    if (!st) {
        for (int i = 0; i < n; ++i)
            b[i] = tau[i] - c[i];
        chol_solve_d(n, L, b, qdd);                                /* qdd = M^-1 (tau - c) */
        st = minv_from_M(n, M, Minv);
    }
    if (!st)
        st = orc_rnea_grad(m, q, qd, qdd, dq, dqd);                /* dtau/du at qdd */
    if (!st) {
        for (int i = 0; i < n; ++i)                                /* dqdd/du = -Minv dtau/du */
            for (int j = 0; j < n; ++j) {
                double s1 = 0, s2 = 0;
                for (int k = 0; k < n; ++k) {
                    s1 += Minv[i * n + k] * dq[k * n + j];
                    s2 += Minv[i * n + k] * dqd[k * n + j];
                }
                dqdd_dq[i * n + j] = -s1;
                dqdd_dqd[i * n + j] = -s2;
            }
    }
    free(M); free(L); free(c); free(zero); free(b); free(dq); free(dqd);
    return st;
}

int orc_fd_grad_batch(const orc_model *m, int N, const double *q, const double *qd,
                      const double *tau, double *qdd, double *Minv, double *dqdd_dq,
                      double *dqdd_dqd)
{
    if (check_model(m) || N < 0)
        return -1;
    const long n = m->n;
    int status = 0;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < N; ++k) {
        int st = orc_fd_grad(m, q + k * n, qd + k * n, tau + k * n, qdd + k * n,
                             Minv + k * n * n, dqdd_dq + k * n * n, dqdd_dqd + k * n * n);
        if (st) {
#pragma omp critical
            if (!status)
                status = st;
        }
    }
    return status;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of later batch calls (timing control only; no effect on any result) */
void orc_set_num_threads(int k)
{
#ifdef _OPENMP
    if (k > 0)
        omp_set_num_threads(k);
#else
    (void)k;
#endif
}
