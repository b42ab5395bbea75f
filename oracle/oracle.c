/*
 * Plain FP64 CPU oracle for the positivity-preserving fifth-order
 * finite-volume compact-WENO (FVCW) scheme for the Euler equations
 * (Guo, Xiong & Shi, arXiv 1402.5618).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent checker that the
 * HIP path is compared against.  It shares no code, header, table or helper
 * with the product library; only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load it.
 *
 * Written for clarity, not speed: every step follows the paper in its order
 * (Sec. 2.1-2.5), component-wise on the conserved variables, in IEEE double
 * with no fast-math and no FMA contraction.  Readings of passages the paper
 * leaves open are marked "reading:" and are listed in the design notes.
 *
 * Layout: a line is [ncomp][n] contiguous; a 2D state is [4][ny][nx];
 * ncomp = 3 (rho, rho u, E) in 1D and 4 (rho, rho u, rho v, E) in 2D.
 * Boundary codes: 0 periodic, 1 transmissive, 2 reflective.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NG 3 /* ghost cells per side for non-periodic lines */

typedef struct {
    double gamma;     /* ratio of specific heats (Sec. 1) */
    double weno_eps;  /* epsilon in the WENO-Z weights, eq. (weight) */
    double eps_cap;   /* cap of the positivity epsilon, limiter step 1 */
    double gl_w1;     /* Gauss-Lobatto end weight w^_1 (= w^_M), Sec. 2.4 */
    int linear;       /* 1: weights forced to (c0,c1,c2): linear scheme, eqs (5th-order1/2) */
    int first_order;  /* 1: no reconstruction, U+- = cell average: scheme (1DEulerFV-First) */
    int limiter;      /* 1: apply the positivity-preserving limiter */
    int flux;         /* 0: HLLC, eq. (HLLC); 1: local Lax-Friedrichs (see lf below) */
    int recon;        /* 0: compact (FVCW, Sec 2.2); 1: explicit WENO-JS; 2: explicit
                       * WENO-Z (the non-compact schemes of Sec 3, see weno5_explicit);
                       * 3: compact, characteristic-wise (Sec 2.3; in 2D along
                       * each line's direction) */
    int fv;           /* 2D face fluxes: 0 one state pair per face (dimension by
                       * dimension); 1 three Gauss-Legendre nodes per face from a
                       * transverse reconstruction (see orc_rhs_2d_gauss) */
} orc_params;

/* Optional per-line intermediate results for tests (any pointer may be NULL). */
typedef struct {
    double *um, *up;       /* [ncomp][n] reconstructed U-_{i+1/2}, U+_{i-1/2} before limiting */
    double *um_l, *up_l;   /* [ncomp][n] after the limiter */
    double *flux;          /* [ncomp][n+1] face fluxes, face f between cells f-1 and f */
} orc_line_dbg;

/* |u_n| + a of a state (normal velocity u_n = U[nrm] / rho).  A pressure
 * that is negative only by roundoff (E almost all kinetic) counts as 0. */
static double wave_speed(double g, int ncomp, int nrm, const double *U)
{
    double m2 = 0.0;
    for (int k = 1; k < ncomp - 1; ++k) m2 += U[k] * U[k];
    double p = (g - 1.0) * (U[ncomp - 1] - 0.5 * m2 / U[0]);
    return fabs(U[nrm] / U[0]) + sqrt(g * fmax(p, 0.0) / U[0]);
}

/* running maximum in which a NaN is sticky */
static void max_into(double *acc, double v)
{
    if (v > *acc || v != v) *acc = v;
}

static double sq(double x) { return x * x; }

/* ------------------------------------------------------------------ Sec 2.2
 * Smoothness indicators of the three candidate stencils of the value at node
 * j+1/2 seen from cell j (the "-" side), from v[0..4] = ubar_{j-2..j+2}.
 * These are the classical indicators printed after eq. (weight). */
static void beta_minus(const double v[5], double b[3])
{
    b[0] = 13.0 / 12.0 * sq(v[0] - 2.0 * v[1] + v[2]) + 0.25 * sq(v[0] - 4.0 * v[1] + 3.0 * v[2]);
    b[1] = 13.0 / 12.0 * sq(v[1] - 2.0 * v[2] + v[3]) + 0.25 * sq(v[1] - v[3]);
    b[2] = 13.0 / 12.0 * sq(v[2] - 2.0 * v[3] + v[4]) + 0.25 * sq(3.0 * v[2] - 4.0 * v[3] + v[4]);
}

/* The "+" side at node j+1/2 (seen from cell j+1) is the mirror image of the
 * "-" side about the node: cell j+m <-> cell j+1-m.  v[0..4] = ubar_{j-1..j+3};
 * candidate k is the mirror of candidate k of the "-" side. */
static void beta_plus(const double v[5], double b[3])
{
    b[0] = 13.0 / 12.0 * sq(v[4] - 2.0 * v[3] + v[2]) + 0.25 * sq(v[4] - 4.0 * v[3] + 3.0 * v[2]);
    b[1] = 13.0 / 12.0 * sq(v[3] - 2.0 * v[2] + v[1]) + 0.25 * sq(v[3] - v[1]);
    b[2] = 13.0 / 12.0 * sq(v[2] - 2.0 * v[1] + v[0]) + 0.25 * sq(3.0 * v[2] - 4.0 * v[1] + v[0]);
}

/* eq. (weight): WENO-Z weights with tau5 = |beta2 - beta0| and power 2. */
static void wenoz(const double b[3], const double c[3], double eps, double w[3])
{
    double tau = fabs(b[2] - b[0]);
    double al[3], s = 0.0;
    for (int k = 0; k < 3; ++k) {
        al[k] = c[k] * (1.0 + sq(tau / (b[k] + eps)));
        s += al[k];
    }
    for (int k = 0; k < 3; ++k) w[k] = al[k] / s;
}

static const double C_LIN[3] = {0.2, 0.5, 0.3}; /* optimal linear weights, Sec 2.2 */

/* Test hook: weights of both sides at node j+1/2 from v[0..5] = ubar_{j-2..j+3}:
 * w[0..2] for the "-" side (cells j-2..j+2), w[3..5] for the "+" side (cells j-1..j+3). */
void orc_weights(const double *v, double eps, double *w)
{
    double b[3];
    beta_minus(v, b);
    wenoz(b, C_LIN, eps, w);
    beta_plus(v + 1, b);
    wenoz(b, C_LIN, eps, w + 3);
}

/* Weights of one side, honouring the "linear" switch. */
static void side_weights(const double b[3], const orc_params *P, double w[3])
{
    if (P->linear) {
        w[0] = C_LIN[0]; w[1] = C_LIN[1]; w[2] = C_LIN[2];
    } else {
        wenoz(b, C_LIN, P->weno_eps, w);
    }
}

/* eq. (CWENO-FV): row at node j+1/2 of the "-" system, coupling
 * u~_{j-1/2}, u~_{j+1/2}, u~_{j+3/2}; right side from ubar_{j-1}, ubar_j, ubar_{j+1}. */
static void row_minus(const double w[3], double um1, double u0, double up1,
                      double *a, double *b, double *c, double *r)
{
    *a = (2.0 * w[0] + w[1]) / 3.0;
    *b = (w[0] + 2.0 * (w[1] + w[2])) / 3.0;
    *c = w[2] / 3.0;
    *r = w[0] / 6.0 * um1 + (5.0 * (w[0] + w[1]) + w[2]) / 6.0 * u0 + (w[1] + 5.0 * w[2]) / 6.0 * up1;
}

/* Mirror of eq. (CWENO-FV) for the "+" system at node j+1/2 (Sec 2.2, last
 * paragraph): coupling u~+_{j-1/2} (a), u~+_{j+1/2} (b), u~+_{j+3/2} (c);
 * right side from ubar_j, ubar_{j+1}, ubar_{j+2}.  With w = c this is eq. (5th-order2). */
static void row_plus(const double w[3], double u0, double up1, double up2,
                     double *a, double *b, double *c, double *r)
{
    *a = w[2] / 3.0;
    *b = (w[0] + 2.0 * (w[1] + w[2])) / 3.0;
    *c = (2.0 * w[0] + w[1]) / 3.0;
    *r = (w[1] + 5.0 * w[2]) / 6.0 * u0 + (5.0 * (w[0] + w[1]) + w[2]) / 6.0 * up1 + w[0] / 6.0 * up2;
}

/* Reading (boundary closure): the nodal value just outside a non-periodic
 * line comes from the classical explicit fifth-order WENO-Z reconstruction on
 * the ghost-extended averages, v[0..4] = ubar_{j-2..j+2}, "-" side of node j+1/2. */
static double weno5z_minus(const double v[5], const orc_params *P)
{
    static const double D5[3] = {0.1, 0.6, 0.3};
    double q0 = (2.0 * v[0] - 7.0 * v[1] + 11.0 * v[2]) / 6.0;
    double q1 = (-v[1] + 5.0 * v[2] + 2.0 * v[3]) / 6.0;
    double q2 = (2.0 * v[2] + 5.0 * v[3] - v[4]) / 6.0;
    double b[3], w[3];
    beta_minus(v, b);
    if (P->linear) { w[0] = D5[0]; w[1] = D5[1]; w[2] = D5[2]; }
    else wenoz(b, D5, P->weno_eps, w);
    return w[0] * q0 + w[1] * q1 + w[2] * q2;
}

/* Sec 3 comparison schemes: the classical explicit fifth-order finite-volume
 * WENO value at node j+1/2 ("-" side) from v[0..4] = ubar_{j-2..j+2}, with
 * the Jiang-Shu weights alpha_k = d_k / (beta_k + eps)^2 (kind 1, eps = 1e-6
 * as in Jiang and Shu's paper: a reading, the paper states none) or the
 * WENO-Z weights of eq. (weight) with d_k in place of c_k (kind 2). */
#define WENO_JS_EPS 1e-6
static double weno5_explicit(const double v[5], int kind, const orc_params *P)
{
    static const double D5[3] = {0.1, 0.6, 0.3};
    if (kind == 2) return weno5z_minus(v, P);
    double q0 = (2.0 * v[0] - 7.0 * v[1] + 11.0 * v[2]) / 6.0;
    double q1 = (-v[1] + 5.0 * v[2] + 2.0 * v[3]) / 6.0;
    double q2 = (2.0 * v[2] + 5.0 * v[3] - v[4]) / 6.0;
    double b[3], al[3], s = 0.0;
    beta_minus(v, b);
    for (int k = 0; k < 3; ++k) {
        al[k] = P->linear ? D5[k] : D5[k] / sq(b[k] + WENO_JS_EPS);
        s += al[k];
    }
    return (al[0] * q0 + al[1] * q1 + al[2] * q2) / s;
}

/* ------------------------------------------------------- tridiagonal solves
 * Chasing (Thomas) elimination, no pivoting: a_i x_{i-1} + b_i x_i + c_i x_{i+1} = r_i,
 * i = 0..n-1, a_0 and c_{n-1} ignored.  Returns 0, or -1 on a zero pivot. */
int orc_thomas(int n, const double *a, const double *b, const double *c, const double *r, double *x)
{
    double *cp = (double *)malloc(sizeof(double) * (size_t)n);
    double *dp = (double *)malloc(sizeof(double) * (size_t)n);
    if (!cp || !dp) { free(cp); free(dp); return -2; }
    int rc = 0;
    if (b[0] == 0.0) { rc = -1; goto done; }
    cp[0] = c[0] / b[0];
    dp[0] = r[0] / b[0];
    for (int i = 1; i < n; ++i) {
        double m = b[i] - a[i] * cp[i - 1];
        if (m == 0.0) { rc = -1; goto done; }
        cp[i] = c[i] / m;
        dp[i] = (r[i] - a[i] * dp[i - 1]) / m;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
done:
    free(cp);
    free(dp);
    return rc;
}

/* Cyclic tridiagonal system (indices mod n, n >= 3): the last unknown is
 * kept as a parameter, x_i = p_i + q_i x_{n-1} from two chasing solves of the
 * leading (n-1)x(n-1) block, then the last row gives x_{n-1}. */
int orc_cyclic(int n, const double *a, const double *b, const double *c, const double *r, double *x)
{
    if (n < 3) return -3;
    int m = n - 1;
    double *v = (double *)calloc((size_t)m, sizeof(double));
    double *p = (double *)malloc(sizeof(double) * (size_t)m);
    double *q = (double *)malloc(sizeof(double) * (size_t)m);
    if (!v || !p || !q) { free(v); free(p); free(q); return -2; }
    v[0] = -a[0];
    v[m - 1] += -c[m - 1];
    int rc = orc_thomas(m, a, b, c, r, p);
    if (rc == 0) rc = orc_thomas(m, a, b, c, v, q);
    if (rc == 0) {
        double den = b[n - 1] + a[n - 1] * q[m - 1] + c[n - 1] * q[0];
        if (den == 0.0) rc = -1;
        else {
            double xl = (r[n - 1] - a[n - 1] * p[m - 1] - c[n - 1] * p[0]) / den;
            for (int i = 0; i < m; ++i) x[i] = p[i] + q[i] * xl;
            x[n - 1] = xl;
        }
    }
    free(v); free(p); free(q);
    return rc;
}

/* Dense Gaussian elimination with partial pivoting on an n x n row-major
 * matrix (test support for small lines).  Returns 0 or -1 if singular. */
int orc_dense_solve(int n, const double *A, const double *r, double *x)
{
    double *M = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(n + 1));
    if (!M) return -2;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) M[i * (n + 1) + j] = A[i * n + j];
        M[i * (n + 1) + n] = r[i];
    }
    int rc = 0;
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(M[i * (n + 1) + k]) > fabs(M[piv * (n + 1) + k])) piv = i;
        if (M[piv * (n + 1) + k] == 0.0) { rc = -1; break; }
        if (piv != k)
            for (int j = 0; j <= n; ++j) {
                double t = M[k * (n + 1) + j];
                M[k * (n + 1) + j] = M[piv * (n + 1) + j];
                M[piv * (n + 1) + j] = t;
            }
        for (int i = k + 1; i < n; ++i) {
            double f = M[i * (n + 1) + k] / M[k * (n + 1) + k];
            for (int j = k; j <= n; ++j) M[i * (n + 1) + j] -= f * M[k * (n + 1) + j];
        }
    }
    if (rc == 0)
        for (int i = n - 1; i >= 0; --i) {
            double s = M[i * (n + 1) + n];
            for (int j = i + 1; j < n; ++j) s -= M[i * (n + 1) + j] * x[j];
            x[i] = s / M[i * (n + 1) + i];
        }
    free(M);
    return rc;
}

/* Reading: the "+" system is chased from its right end, the mirror of the
 * "-" sweep: solve on the reversed system (a and c exchange roles). */
static int solve_reversed(int n, int cyclic, const double *a, const double *b, const double *c,
                          const double *r, double *x, double *work /* 5n */)
{
    double *ra = work, *rb = work + n, *rc = work + 2 * n, *rr = work + 3 * n, *rx = work + 4 * n;
    for (int i = 0; i < n; ++i) {
        ra[i] = c[n - 1 - i];
        rb[i] = b[n - 1 - i];
        rc[i] = a[n - 1 - i];
        rr[i] = r[n - 1 - i];
    }
    int s = cyclic ? orc_cyclic(n, ra, rb, rc, rr, rx) : orc_thomas(n, ra, rb, rc, rr, rx);
    for (int i = 0; i < n; ++i) x[i] = rx[n - 1 - i];
    return s;
}

/* -------------------------------------------------------------- Sec 2.2-2.3
 * Component-wise reconstruction of one scalar line.  ue[0..n+5] holds the
 * averages of cells -3..n+2 (cell i at ue[i+3]); for a periodic line the
 * ghosts are the wrapped cells.  Outputs: um[i] = u-_{i+1/2} (right face of
 * cell i, "-" system) and up[i] = u+_{i-1/2} (left face of cell i, "+" system). */
static int recon_scalar(int n, int cyclic, const double *ue, const orc_params *P,
                        double *um, double *up, double *work /* >= 9n */)
{
    double *a = work, *b = work + n, *c = work + 2 * n, *r = work + 3 * n;
    double *w5 = work + 4 * n;
    double v[5], beta[3], w[3];
    if (P->recon != 0) {
        /* explicit schemes: each face value from its own five averages; the
         * "+" value at node i-1/2 is the "-" formula on the stencil mirrored
         * about that node (cells i+2 .. i-2) */
        for (int i = 0; i < n; ++i) {
            for (int k = 0; k < 5; ++k) v[k] = ue[i + 1 + k];
            um[i] = weno5_explicit(v, P->recon, P);
            for (int k = 0; k < 5; ++k) v[k] = ue[i + 5 - k];
            up[i] = weno5_explicit(v, P->recon, P);
        }
        return 0;
    }
    /* "-" system: row i sits at node i+1/2; stencil cells i-2..i+2. */
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < 5; ++k) v[k] = ue[i + 1 + k];
        beta_minus(v, beta);
        side_weights(beta, P, w);
        row_minus(w, v[1], v[2], v[3], &a[i], &b[i], &c[i], &r[i]);
    }
    int s;
    if (cyclic) {
        s = orc_cyclic(n, a, b, c, r, um);
    } else {
        /* closure values u-_{-1/2} (cell -1) and u-_{n+1/2} (cell n) */
        double xl = weno5z_minus(&ue[0], P);
        double xr = weno5z_minus(&ue[n + 1], P);
        r[0] -= a[0] * xl;
        r[n - 1] -= c[n - 1] * xr;
        s = orc_thomas(n, a, b, c, r, um);
    }
    if (s) return s;
    /* "+" system: unknown i is u+ at node i-1/2; its row is the mirrored row at
     * that node, with stencil cells i-2..i+2 (right side from i-1, i, i+1). */
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < 5; ++k) v[k] = ue[i + 1 + k];
        beta_plus(v, beta);
        side_weights(beta, P, w);
        row_plus(w, v[1], v[2], v[3], &a[i], &b[i], &c[i], &r[i]);
    }
    if (cyclic) {
        s = solve_reversed(n, 1, a, b, c, r, up, w5);
    } else {
        /* closure values u+ at the left faces of cells -1 and n: mirrored
         * explicit reconstruction on the reversed stencils */
        double mv[5];
        for (int k = 0; k < 5; ++k) mv[k] = ue[4 - k];     /* cells 1..-3 */
        double xl = weno5z_minus(mv, P);
        for (int k = 0; k < 5; ++k) mv[k] = ue[n + 5 - k]; /* cells n+2..n-2 */
        double xr = weno5z_minus(mv, P);
        r[0] -= a[0] * xl;
        r[n - 1] -= c[n - 1] * xr;
        s = solve_reversed(n, 0, a, b, c, r, up, w5);
    }
    return s;
}

/* ----------------------------------------------------------------- Sec 2.3
 * Characteristic-wise compact reconstruction of the 1D Euler system
 * (recon = 3): at each node the scalar rows of eq. (CWENO-FV) are formed per
 * characteristic field from the characteristic variables l^(k) . Ubar of the
 * Roe average at that node, and stacked into the 3x3 block tridiagonal
 * system (1DEuler-FVC) in the conserved nodal values, solved by block
 * chasing.  The 2D operator applies the same construction line by line
 * (dimension by dimension), with the eigenvectors of the flux Jacobian
 * along the line: 4x4 blocks. */

/* Roe average of the states Ua, Ub (rho, rho u, E) and, there, the left
 * eigenvectors l^(k) (rows of L, eq. (leigenv)), the right eigenvectors
 * r^(k) (columns of R, eq. (reigenv)) and the eigenvalues (eq. (eigen)).
 * Reading: a Roe sound speed that is not positive (two states without
 * pressure moving together) makes the node component-wise (L = R = I). */
static void roe_eigen(double g, const double *Ua, const double *Ub, double L[3][3],
                      double R[3][3], double lam[3])
{
    double ra = Ua[0], rb = Ub[0];
    double ua = Ua[1] / ra, ub = Ub[1] / rb;
    double pa = (g - 1.0) * (Ua[2] - 0.5 * ra * ua * ua);
    double pb = (g - 1.0) * (Ub[2] - 0.5 * rb * ub * ub);
    double Ha = (Ua[2] + pa) / ra, Hb = (Ub[2] + pb) / rb;
    double sa = sqrt(ra), sb = sqrt(rb);
    double u = (sa * ua + sb * ub) / (sa + sb);
    double H = (sa * Ha + sb * Hb) / (sa + sb);
    double a2 = (g - 1.0) * (H - 0.5 * u * u);
    if (!(a2 > 0.0)) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) L[i][j] = R[i][j] = (i == j) ? 1.0 : 0.0;
        lam[0] = lam[1] = lam[2] = u;
        return;
    }
    double a = sqrt(a2);
    double c1 = (g - 1.0) / a2, c2 = 0.5 * u * u * c1;
    L[0][0] = 0.5 * (c2 + u / a); L[0][1] = 0.5 * (-c1 * u - 1.0 / a); L[0][2] = 0.5 * c1;
    L[1][0] = 1.0 - c2;           L[1][1] = c1 * u;                    L[1][2] = -c1;
    L[2][0] = 0.5 * (c2 - u / a); L[2][1] = 0.5 * (-c1 * u + 1.0 / a); L[2][2] = 0.5 * c1;
    R[0][0] = 1.0;         R[0][1] = 1.0;           R[0][2] = 1.0;
    R[1][0] = u - a;       R[1][1] = u;             R[1][2] = u + a;
    R[2][0] = H - u * a;   R[2][1] = 0.5 * u * u;   R[2][2] = H + u * a;
    lam[0] = u - a; lam[1] = u; lam[2] = u + a;
}

/* Exported for unit tests: L and R row-major [3][3]. */
void orc_char_eigen(double gamma, const double *Ua, const double *Ub, double *Lo, double *Ro,
                    double *lam)
{
    double L[3][3], R[3][3];
    roe_eigen(gamma, Ua, Ub, L, R, lam);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) { Lo[3 * i + j] = L[i][j]; Ro[3 * i + j] = R[i][j]; }
}

/* The 2D form, for a line of the dimension-by-dimension extension: Roe
 * average of Ua, Ub (rho, rho u, rho v, E) and the eigenvectors of the flux
 * Jacobian along the line, whose normal momentum is component nrm (1: x,
 * 2: y; t = 3 - nrm is the tangential one).  With q^2 = u_n^2 + u_t^2,
 * b1 = (gamma-1)/a^2 and b2 = b1 q^2 / 2 the fields are, in this order, the
 * acoustic wave u_n - a, the entropy wave u_n, the shear wave u_n (which
 * carries u_t) and the acoustic wave u_n + a:
 *   l0 = ( b2 + u_n/a, -b1 u_n - 1/a, -b1 u_t, b1 ) / 2   r0 = (1, u_n - a, u_t, H - u_n a)
 *   l1 = ( 1 - b2,      b1 u_n,        b1 u_t, -b1 )      r1 = (1, u_n,     u_t, q^2/2)
 *   l2 = ( -u_t,        0,             1,       0  )      r2 = (0, 0,       1,   u_t)
 *   l3 = ( b2 - u_n/a, -b1 u_n + 1/a, -b1 u_t, b1 ) / 2   r3 = (1, u_n + a, u_t, H + u_n a)
 * (entries listed in the order rho, normal momentum, tangential momentum,
 * E).  With u_t = 0 the acoustic and entropy fields are those of the 1D
 * system and the shear field is the tangential momentum itself.  The same
 * reading as in 1D for a Roe sound speed that is not positive. */
static void roe_eigen2(double g, int nrm, const double *Ua, const double *Ub, double L[4][4],
                       double R[4][4], double lam[4])
{
    int t = 3 - nrm;
    double ra = Ua[0], rb = Ub[0];
    double una = Ua[nrm] / ra, unb = Ub[nrm] / rb;
    double uta = Ua[t] / ra, utb = Ub[t] / rb;
    double pa = (g - 1.0) * (Ua[3] - 0.5 * ra * (una * una + uta * uta));
    double pb = (g - 1.0) * (Ub[3] - 0.5 * rb * (unb * unb + utb * utb));
    double Ha = (Ua[3] + pa) / ra, Hb = (Ub[3] + pb) / rb;
    double sa = sqrt(ra), sb = sqrt(rb);
    double un = (sa * una + sb * unb) / (sa + sb);
    double ut = (sa * uta + sb * utb) / (sa + sb);
    double H = (sa * Ha + sb * Hb) / (sa + sb);
    double q2 = un * un + ut * ut;
    double a2 = (g - 1.0) * (H - 0.5 * q2);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) L[i][j] = R[i][j] = 0.0;
    if (!(a2 > 0.0)) {
        for (int i = 0; i < 4; ++i) { L[i][i] = R[i][i] = 1.0; lam[i] = un; }
        return;
    }
    double a = sqrt(a2);
    double b1 = (g - 1.0) / a2, b2 = 0.5 * q2 * b1;
    L[0][0] = 0.5 * (b2 + un / a); L[0][nrm] = 0.5 * (-b1 * un - 1.0 / a);
    L[0][t] = -0.5 * b1 * ut;      L[0][3] = 0.5 * b1;
    L[1][0] = 1.0 - b2;            L[1][nrm] = b1 * un;
    L[1][t] = b1 * ut;             L[1][3] = -b1;
    L[2][0] = -ut;                 L[2][t] = 1.0;
    L[3][0] = 0.5 * (b2 - un / a); L[3][nrm] = 0.5 * (-b1 * un + 1.0 / a);
    L[3][t] = -0.5 * b1 * ut;      L[3][3] = 0.5 * b1;
    R[0][0] = 1.0; R[nrm][0] = un - a; R[t][0] = ut; R[3][0] = H - un * a;
    R[0][1] = 1.0; R[nrm][1] = un;     R[t][1] = ut; R[3][1] = 0.5 * q2;
    R[t][2] = 1.0; R[3][2] = ut;
    R[0][3] = 1.0; R[nrm][3] = un + a; R[t][3] = ut; R[3][3] = H + un * a;
    lam[0] = un - a; lam[1] = un; lam[2] = un; lam[3] = un + a;
}

/* Exported for unit tests: L and R row-major [4][4]. */
void orc_char_eigen2(double gamma, int nrm, const double *Ua, const double *Ub, double *Lo,
                     double *Ro, double *lam)
{
    double L[4][4], R[4][4];
    roe_eigen2(gamma, nrm, Ua, Ub, L, R, lam);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) { Lo[4 * i + j] = L[i][j]; Ro[4 * i + j] = R[i][j]; }
}

/* Blocks of nb x nb (nb = 3 in 1D, 4 in 2D), row-major and flat. */
#define NBMAX 4

/* Solve M X = Y for an nb x nb M and k right-hand columns (Y, X row-major
 * nb x k, k <= 2 nb + 1), Gaussian elimination with partial pivoting.
 * Returns 0 or -1 if singular. */
static int solve_nb(int nb, const double *M, int k, const double *Y, double *X)
{
    double T[NBMAX][3 * NBMAX + 1];
    for (int i = 0; i < nb; ++i) {
        for (int j = 0; j < nb; ++j) T[i][j] = M[i * nb + j];
        for (int j = 0; j < k; ++j) T[i][nb + j] = Y[i * k + j];
    }
    for (int c = 0; c < nb; ++c) {
        int piv = c;
        for (int i = c + 1; i < nb; ++i)
            if (fabs(T[i][c]) > fabs(T[piv][c])) piv = i;
        if (T[piv][c] == 0.0) return -1;
        if (piv != c)
            for (int j = 0; j < nb + k; ++j) { double t = T[c][j]; T[c][j] = T[piv][j]; T[piv][j] = t; }
        for (int i = c + 1; i < nb; ++i) {
            double f = T[i][c] / T[c][c];
            for (int j = c; j < nb + k; ++j) T[i][j] -= f * T[c][j];
        }
    }
    for (int j = 0; j < k; ++j)
        for (int i = nb - 1; i >= 0; --i) {
            double v = T[i][nb + j];
            for (int l = i + 1; l < nb; ++l) v -= T[i][l] * X[l * k + j];
            X[i * k + j] = v / T[i][i];
        }
    return 0;
}

/* Y -= M X for an nb x nb M and X, Y of k columns (row-major nb x k). */
static void sub_mul_nb(int nb, const double *M, int k, const double *X, double *Y)
{
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < k; ++j)
            for (int l = 0; l < nb; ++l) Y[i * k + j] -= M[i * nb + l] * X[l * k + j];
}

/* Block chasing (the paper's method for (1DEuler-FVC)):
 * A_i X_{i-1} + B_i X_i + C_i X_{i+1} = Y_i, i = 0..n-1, nb x nb blocks
 * ([n][nb][nb]; A_0 and C_{n-1} ignored), Y_i and X_i of k <= nb + 1 columns
 * ([n][nb][k]).  Block LU without pivoting between blocks; each pivot block
 * solved with partial pivoting.  Returns 0, -1 on a singular pivot block,
 * -2 on no memory. */
static int blk_thomas(int nb, int n, int k, const double *A, const double *B, const double *C,
                      const double *Y, double *X)
{
    size_t bb = (size_t)nb * (size_t)nb, bk = (size_t)nb * (size_t)k;
    double *Cp = (double *)malloc(sizeof(double) * bb * (size_t)n);
    double *Dp = (double *)malloc(sizeof(double) * bk * (size_t)n);
    if (!Cp || !Dp) { free(Cp); free(Dp); return -2; }
    int rc = 0, w = nb + k;
    for (int i = 0; i < n && rc == 0; ++i) {
        double M[NBMAX * NBMAX], rhs[NBMAX * (2 * NBMAX + 1)], sol[NBMAX * (2 * NBMAX + 1)];
        const double *Ai = A + (size_t)i * bb, *Bi = B + (size_t)i * bb, *Ci = C + (size_t)i * bb;
        for (int r = 0; r < nb; ++r)
            for (int c = 0; c < nb; ++c) M[r * nb + c] = Bi[r * nb + c];
        for (int r = 0; r < nb; ++r) {
            for (int c = 0; c < nb; ++c) rhs[r * w + c] = (i < n - 1) ? Ci[r * nb + c] : 0.0;
            for (int c = 0; c < k; ++c) rhs[r * w + nb + c] = Y[(size_t)i * bk + r * k + c];
        }
        if (i > 0) {
            /* M = B_i - A_i Cp_{i-1};  rhs(Y part) -= A_i Dp_{i-1} */
            const double *Cq = Cp + (size_t)(i - 1) * bb, *Dq = Dp + (size_t)(i - 1) * bk;
            for (int r = 0; r < nb; ++r)
                for (int c = 0; c < nb; ++c)
                    for (int l = 0; l < nb; ++l) M[r * nb + c] -= Ai[r * nb + l] * Cq[l * nb + c];
            for (int r = 0; r < nb; ++r)
                for (int c = 0; c < k; ++c)
                    for (int l = 0; l < nb; ++l) rhs[r * w + nb + c] -= Ai[r * nb + l] * Dq[l * k + c];
        }
        rc = solve_nb(nb, M, w, rhs, sol);
        for (int r = 0; r < nb; ++r) {
            for (int c = 0; c < nb; ++c) Cp[(size_t)i * bb + r * nb + c] = sol[r * w + c];
            for (int c = 0; c < k; ++c) Dp[(size_t)i * bk + r * k + c] = sol[r * w + nb + c];
        }
    }
    if (rc == 0) {
        for (size_t j = 0; j < bk; ++j) X[(size_t)(n - 1) * bk + j] = Dp[(size_t)(n - 1) * bk + j];
        for (int i = n - 2; i >= 0; --i) {
            for (size_t j = 0; j < bk; ++j) X[(size_t)i * bk + j] = Dp[(size_t)i * bk + j];
            sub_mul_nb(nb, Cp + (size_t)i * bb, k, &X[(size_t)(i + 1) * bk], &X[(size_t)i * bk]);
        }
    }
    free(Cp);
    free(Dp);
    return rc;
}

/* Block cyclic system (indices mod n, n >= 3), one right-hand column: the
 * last unknown is kept as a parameter, X_i = P_i + Q_i X_{n-1} from the
 * leading (n-1) block rows (right-hand columns Y and the two coupling
 * blocks), then the last block row gives X_{n-1}. */
static int blk_cyclic(int nb, int n, const double *A, const double *B, const double *C,
                      const double *Y, double *X)
{
    int m = n - 1, K = nb + 1;
    size_t bb = (size_t)nb * (size_t)nb, bK = (size_t)nb * (size_t)K;
    double *Y4 = (double *)calloc((size_t)m * bK, sizeof(double));
    double *S4 = (double *)malloc(sizeof(double) * (size_t)m * bK);
    if (!Y4 || !S4) { free(Y4); free(S4); return -2; }
    for (int i = 0; i < m; ++i)
        for (int r = 0; r < nb; ++r) Y4[(size_t)i * bK + r * K] = Y[nb * i + r];
    for (int r = 0; r < nb; ++r)
        for (int c = 0; c < nb; ++c) {
            Y4[r * K + 1 + c] -= A[r * nb + c];                                   /* row 0 couples X_{n-1} */
            Y4[(size_t)(m - 1) * bK + r * K + 1 + c] -= C[(size_t)(m - 1) * bb + r * nb + c];  /* row n-2 too */
        }
    int rc = blk_thomas(nb, m, K, A, B, C, Y4, S4);
    if (rc == 0) {
        /* (B_{n-1} + A_{n-1} Q_{n-2} + C_{n-1} Q_0) X_{n-1} = Y_{n-1} - A_{n-1} P_{n-2} - C_{n-1} P_0 */
        double M[NBMAX * NBMAX], rhs[NBMAX], xl[NBMAX];
        const double *Sl = &S4[(size_t)(m - 1) * bK], *S0 = &S4[0];
        const double *Al = A + (size_t)(n - 1) * bb, *Bl = B + (size_t)(n - 1) * bb,
                     *Cl = C + (size_t)(n - 1) * bb;
        for (int r = 0; r < nb; ++r) {
            rhs[r] = Y[nb * (n - 1) + r];
            for (int c = 0; c < nb; ++c) {
                M[r * nb + c] = Bl[r * nb + c];
                for (int l = 0; l < nb; ++l)
                    M[r * nb + c] += Al[r * nb + l] * Sl[l * K + 1 + c] + Cl[r * nb + l] * S0[l * K + 1 + c];
            }
            for (int l = 0; l < nb; ++l)
                rhs[r] -= Al[r * nb + l] * Sl[l * K] + Cl[r * nb + l] * S0[l * K];
        }
        rc = solve_nb(nb, M, 1, rhs, xl);
        if (rc == 0) {
            for (int i = 0; i < m; ++i)
                for (int r = 0; r < nb; ++r) {
                    double v = S4[(size_t)i * bK + r * K];
                    for (int c = 0; c < nb; ++c) v += S4[(size_t)i * bK + r * K + 1 + c] * xl[c];
                    X[nb * i + r] = v;
                }
            for (int r = 0; r < nb; ++r) X[nb * (n - 1) + r] = xl[r];
        }
    }
    free(Y4);
    free(S4);
    return rc;
}

/* Exported for unit tests: A, B, C [n][nb][nb], Y, X [n][nb], nb = 3 or 4. */
int orc_block_solve_nb(int nb, int n, int cyclic, const double *A, const double *B,
                       const double *C, const double *Y, double *X)
{
    if (nb < 1 || nb > NBMAX) return -3;
    if (cyclic) {
        if (n < 3) return -3;
        return blk_cyclic(nb, n, A, B, C, Y, X);
    }
    return blk_thomas(nb, n, 1, A, B, C, Y, X);
}

/* The 3x3 form (1D). */
int orc_block_solve(int n, int cyclic, const double *A, const double *B, const double *C,
                    const double *Y, double *X)
{
    return orc_block_solve_nb(3, n, cyclic, A, B, C, Y, X);
}

/* The characteristic-wise reconstruction of one line of nb = 3 (1D) or 4
 * (2D, normal momentum component nrm) components: ue [nb][n+6] holds the
 * ghost-extended averages (cell i at ue[c][i+3]).  um[c][i] = U-_{i+1/2},
 * up[c][i] = U+_{i-1/2}.  Rows of the "-" system sit at node i+1/2 with the
 * eigenvectors of Roe(Ubar_i, Ubar_{i+1}); rows of the "+" system at node
 * i-1/2 with those of Roe(Ubar_{i-1}, Ubar_i), the mirrored rows of Sec. 2.2,
 * chased from the right end.  Non-periodic lines are closed as the
 * component-wise ones (reading R10). */
static int recon_char(int nb, int nrm, int n, int cyclic, const double *ue, const orc_params *P,
                      double *um, double *up)
{
    int ne = n + 2 * NG;
    size_t bb = (size_t)nb * (size_t)nb;
    double *A = (double *)malloc(sizeof(double) * 3u * bb * (size_t)n);
    double *Bm = A ? A + bb * (size_t)n : NULL, *Cm = A ? A + 2 * bb * (size_t)n : NULL;
    double *Y = (double *)malloc(sizeof(double) * 2u * (size_t)nb * (size_t)n);
    double *X = Y ? Y + (size_t)nb * n : NULL;
    if (!A || !Y) { free(A); free(Y); return -2; }
#define UE(c, m) ue[(size_t)(c) * ne + (m) + NG]
    for (int side = 0; side < 2; ++side) {
        for (int i = 0; i < n; ++i) {
            double Ua[NBMAX], Ub[NBMAX], L[NBMAX][NBMAX];
            int ca = side == 0 ? i : i - 1;   /* Roe pair of the row's node */
            for (int c = 0; c < nb; ++c) { Ua[c] = UE(c, ca); Ub[c] = UE(c, ca + 1); }
            if (nb == 3) {
                double L3[3][3], R3[3][3], lam[3];
                roe_eigen(P->gamma, Ua, Ub, L3, R3, lam);
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) L[r][c] = L3[r][c];
            } else {
                double R4[4][4], lam[4];
                roe_eigen2(P->gamma, nrm, Ua, Ub, L, R4, lam);
            }
            for (int k = 0; k < nb; ++k) {
                double v[5], beta[3], w[3], a, b, c, r;
                for (int m = 0; m < 5; ++m) {
                    v[m] = 0.0;
                    for (int q = 0; q < nb; ++q) v[m] += L[k][q] * UE(q, i - 2 + m);
                }
                if (side == 0) {
                    beta_minus(v, beta);
                    side_weights(beta, P, w);
                    row_minus(w, v[1], v[2], v[3], &a, &b, &c, &r);
                } else {
                    beta_plus(v, beta);
                    side_weights(beta, P, w);
                    row_plus(w, v[1], v[2], v[3], &a, &b, &c, &r);
                }
                for (int q = 0; q < nb; ++q) {
                    A[(size_t)i * bb + k * nb + q] = a * L[k][q];
                    Bm[(size_t)i * bb + k * nb + q] = b * L[k][q];
                    Cm[(size_t)i * bb + k * nb + q] = c * L[k][q];
                }
                Y[(size_t)nb * i + k] = r;
            }
        }
        int s;
        const double *A0 = A, *Cl = Cm + (size_t)(n - 1) * bb;
        if (side == 0) {
            if (cyclic) {
                s = blk_cyclic(nb, n, A, Bm, Cm, Y, X);
            } else {
                /* closure values U-_{-1/2} (cell -1) and U-_{n+1/2} (cell n) */
                double xl[NBMAX], xr[NBMAX];
                for (int c = 0; c < nb; ++c) {
                    xl[c] = weno5z_minus(&ue[(size_t)c * ne + 0], P);
                    xr[c] = weno5z_minus(&ue[(size_t)c * ne + n + 1], P);
                }
                for (int k = 0; k < nb; ++k)
                    for (int q = 0; q < nb; ++q) {
                        Y[k] -= A0[k * nb + q] * xl[q];
                        Y[(size_t)nb * (n - 1) + k] -= Cl[k * nb + q] * xr[q];
                    }
                s = blk_thomas(nb, n, 1, A, Bm, Cm, Y, X);
            }
            for (int i = 0; i < n && s == 0; ++i)
                for (int c = 0; c < nb; ++c) um[(size_t)c * n + i] = X[(size_t)nb * i + c];
        } else {
            if (!cyclic) {
                /* closure values U+ at the left faces of cells -1 and n */
                double xl[NBMAX], xr[NBMAX], mv[5];
                for (int c = 0; c < nb; ++c) {
                    for (int k = 0; k < 5; ++k) mv[k] = ue[(size_t)c * ne + 4 - k];
                    xl[c] = weno5z_minus(mv, P);
                    for (int k = 0; k < 5; ++k) mv[k] = ue[(size_t)c * ne + n + 5 - k];
                    xr[c] = weno5z_minus(mv, P);
                }
                for (int k = 0; k < nb; ++k)
                    for (int q = 0; q < nb; ++q) {
                        Y[k] -= A0[k * nb + q] * xl[q];
                        Y[(size_t)nb * (n - 1) + k] -= Cl[k * nb + q] * xr[q];
                    }
            }
            /* chased from the right end: the reversed system, A and C exchanged */
            double *rA = (double *)malloc(sizeof(double) * 3u * bb * (size_t)n);
            double *rY = (double *)malloc(sizeof(double) * 2u * (size_t)nb * (size_t)n);
            if (!rA || !rY) { free(rA); free(rY); s = -2; }
            else {
                double *rB = rA + bb * (size_t)n, *rC = rA + 2 * bb * (size_t)n;
                double *rX = rY + (size_t)nb * n;
                for (int i = 0; i < n; ++i) {
                    int j = n - 1 - i;
                    for (size_t q = 0; q < bb; ++q) {
                        rA[(size_t)i * bb + q] = Cm[(size_t)j * bb + q];
                        rB[(size_t)i * bb + q] = Bm[(size_t)j * bb + q];
                        rC[(size_t)i * bb + q] = A[(size_t)j * bb + q];
                    }
                    for (int k = 0; k < nb; ++k) rY[(size_t)nb * i + k] = Y[(size_t)nb * j + k];
                }
                s = cyclic ? blk_cyclic(nb, n, rA, rB, rC, rY, rX)
                           : blk_thomas(nb, n, 1, rA, rB, rC, rY, rX);
                for (int i = 0; i < n && s == 0; ++i)
                    for (int c = 0; c < nb; ++c)
                        up[(size_t)c * n + (n - 1 - i)] = rX[(size_t)nb * i + c];
                free(rA);
                free(rY);
            }
        }
        if (s) { free(A); free(Y); return s; }
    }
#undef UE
    free(A);
    free(Y);
    return 0;
}

/* Exported for unit tests: ue [3][n+6] ghost-extended averages (1D). */
int orc_recon_char(int n, int cyclic, const double *ue, const orc_params *P, double *um, double *up)
{
    return recon_char(3, 1, n, cyclic, ue, P, um, up);
}

/* The 2D form: ue [4][n+6], a line whose normal momentum is component nrm. */
int orc_recon_char2(int nrm, int n, int cyclic, const double *ue, const orc_params *P,
                    double *um, double *up)
{
    if (nrm != 1 && nrm != 2) return -3;
    return recon_char(4, nrm, n, cyclic, ue, P, um, up);
}

/* ----------------------------------------------------------------- Sec 2.4
 * HLLC flux (eqs. (HLLC), (contact-v), (star-l), (acoustic ws)) across a
 * face whose normal momentum is component `nrm` (1: x, 2: y).
 * Readings: the contact speed denominator uses rho_r for the right state and
 * S_R takes the max of its two candidates (the printed formulas repeat
 * rho_l and write min).  In 2D the tangential momentum of a star state is
 * rho* times the tangential velocity of its side.  Sound speeds use
 * max(p, 0): the limiter leaves interface states with e = eps, whose
 * pressure computed from (rho, m, E) is pure roundoff and may come out
 * slightly negative; the Roe sound-speed argument is clipped likewise. */
static void hllc(double g, int ncomp, int nrm, const double *Ul, const double *Ur, double *F)
{
    int ie = ncomp - 1, tg = (ncomp == 4) ? 3 - nrm : -1;
    double rl = Ul[0], ul = Ul[nrm] / rl, vl = tg > 0 ? Ul[tg] / rl : 0.0, El = Ul[ie];
    double rr = Ur[0], ur = Ur[nrm] / rr, vr = tg > 0 ? Ur[tg] / rr : 0.0, Er = Ur[ie];
    double pl = (g - 1.0) * (El - 0.5 * rl * (ul * ul + vl * vl));
    double pr = (g - 1.0) * (Er - 0.5 * rr * (ur * ur + vr * vr));
    double al = sqrt(g * fmax(pl, 0.0) / rl), ar = sqrt(g * fmax(pr, 0.0) / rr);
    double Hl = (El + pl) / rl, Hr = (Er + pr) / rr;
    double R = sqrt(rr / rl);
    double ut = (ul + ur * R) / (1.0 + R);
    double vt = (vl + vr * R) / (1.0 + R);
    double Ht = (Hl + Hr * R) / (1.0 + R);
    double at = sqrt(fmax((g - 1.0) * (Ht - 0.5 * (ut * ut + vt * vt)), 0.0));
    double SL = fmin(ul - al, ut - at);
    double SR = fmax(ur + ar, ut + at);
    /* reading: the denominator is >= 0; it vanishes only when two states
     * with zero computed sound speed separate, and then the midpoint makes
     * both star states vacuum (zero flux), the limit of a -> 0+ */
    double den = rr * (SR - ur) - rl * (SL - ul);
    double SM = den > 0.0 ? (rr * ur * (SR - ur) - rl * ul * (SL - ul) + pl - pr) / den
                          : 0.5 * (SL + SR);
    double Fl[4], Fr[4];
    Fl[0] = rl * ul; Fl[nrm] = rl * ul * ul + pl; Fl[ie] = ul * (El + pl);
    Fr[0] = rr * ur; Fr[nrm] = rr * ur * ur + pr; Fr[ie] = ur * (Er + pr);
    if (tg > 0) { Fl[tg] = rl * ul * vl; Fr[tg] = rr * ur * vr; }
    if (SL > 0.0) {
        for (int k = 0; k < ncomp; ++k) F[k] = Fl[k];
    } else if (SM > 0.0) {
        double d = SL - SM, ps = rl * (ul - SL) * (ul - SM) + pl, Us[4];
        Us[0] = rl * (SL - ul) / d;
        Us[nrm] = ((SL - ul) * rl * ul + (ps - pl)) / d;
        Us[ie] = ((SL - ul) * El - pl * ul + ps * SM) / d;
        if (tg > 0) Us[tg] = Us[0] * vl;
        for (int k = 0; k < ncomp; ++k) F[k] = Fl[k] + SL * (Us[k] - Ul[k]);
    } else if (SR >= 0.0 && SR > SM) {
        double d = SR - SM, ps = rr * (ur - SR) * (ur - SM) + pr, Us[4];
        Us[0] = rr * (SR - ur) / d;
        Us[nrm] = ((SR - ur) * rr * ur + (ps - pr)) / d;
        Us[ie] = ((SR - ur) * Er - pr * ur + ps * SM) / d;
        if (tg > 0) Us[tg] = Us[0] * vr;
        for (int k = 0; k < ncomp; ++k) F[k] = Fr[k] + SR * (Us[k] - Ur[k]);
    } else {
        for (int k = 0; k < ncomp; ++k) F[k] = Fr[k];
    }
}

/* Lax-Friedrichs flux, which the paper names (Example 3.6) as a more
 * dissipative alternative to HLLC without defining it.  Reading: the local
 * form, F = (f(Ul) + f(Ur))/2 - alpha (Ur - Ul)/2 with alpha the larger of
 * |u| + a over the two states; sound speeds from max(p, 0) as in HLLC. */
static void lf(double g, int ncomp, int nrm, const double *Ul, const double *Ur, double *F)
{
    int ie = ncomp - 1, tg = (ncomp == 4) ? 3 - nrm : -1;
    double rl = Ul[0], ul = Ul[nrm] / rl, vl = tg > 0 ? Ul[tg] / rl : 0.0, El = Ul[ie];
    double rr = Ur[0], ur = Ur[nrm] / rr, vr = tg > 0 ? Ur[tg] / rr : 0.0, Er = Ur[ie];
    double pl = (g - 1.0) * (El - 0.5 * rl * (ul * ul + vl * vl));
    double pr = (g - 1.0) * (Er - 0.5 * rr * (ur * ur + vr * vr));
    double al = sqrt(g * fmax(pl, 0.0) / rl), ar = sqrt(g * fmax(pr, 0.0) / rr);
    double alpha = fmax(fabs(ul) + al, fabs(ur) + ar);
    double Fl[4], Fr[4];
    Fl[0] = rl * ul; Fl[nrm] = rl * ul * ul + pl; Fl[ie] = ul * (El + pl);
    Fr[0] = rr * ur; Fr[nrm] = rr * ur * ur + pr; Fr[ie] = ur * (Er + pr);
    if (tg > 0) { Fl[tg] = rl * ul * vl; Fr[tg] = rr * ur * vr; }
    for (int k = 0; k < ncomp; ++k) F[k] = 0.5 * (Fl[k] + Fr[k]) - 0.5 * alpha * (Ur[k] - Ul[k]);
}

/* Exported for unit tests. */
void orc_lf(double gamma, int ncomp, int nrm, const double *Ul, const double *Ur, double *F)
{
    lf(gamma, ncomp, nrm, Ul, Ur, F);
}

/* Exported for unit tests. */
void orc_hllc(double gamma, int ncomp, int nrm, const double *Ul, const double *Ur, double *F)
{
    hllc(gamma, ncomp, nrm, Ul, Ur, F);
}

/* HLLC wave-speed estimates and contact speed, for tests of eq. (inequ-v). */
void orc_hllc_speeds(double g, int ncomp, int nrm, const double *Ul, const double *Ur, double *S)
{
    int ie = ncomp - 1, tg = (ncomp == 4) ? 3 - nrm : -1;
    double rl = Ul[0], ul = Ul[nrm] / rl, vl = tg > 0 ? Ul[tg] / rl : 0.0, El = Ul[ie];
    double rr = Ur[0], ur = Ur[nrm] / rr, vr = tg > 0 ? Ur[tg] / rr : 0.0, Er = Ur[ie];
    double pl = (g - 1.0) * (El - 0.5 * rl * (ul * ul + vl * vl));
    double pr = (g - 1.0) * (Er - 0.5 * rr * (ur * ur + vr * vr));
    double al = sqrt(g * fmax(pl, 0.0) / rl), ar = sqrt(g * fmax(pr, 0.0) / rr);
    double Hl = (El + pl) / rl, Hr = (Er + pr) / rr;
    double R = sqrt(rr / rl);
    double ut = (ul + ur * R) / (1.0 + R), vt = (vl + vr * R) / (1.0 + R);
    double Ht = (Hl + Hr * R) / (1.0 + R);
    double at = sqrt(fmax((g - 1.0) * (Ht - 0.5 * (ut * ut + vt * vt)), 0.0));
    S[0] = fmin(ul - al, ut - at);
    S[2] = fmax(ur + ar, ut + at);
    double den = rr * (S[2] - ur) - rl * (S[0] - ul);
    S[1] = den > 0.0 ? (rr * ur * (S[2] - ur) - rl * ul * (S[0] - ul) + pl - pr) / den
                     : 0.5 * (S[0] + S[2]);
}

/* Specific internal energy e = E/rho - |m|^2/(2 rho^2) (definition of G). */
static double spec_e(int ncomp, const double *U)
{
    double m2 = 0.0;
    for (int k = 1; k < ncomp - 1; ++k) m2 += U[k] * U[k];
    return U[ncomp - 1] / U[0] - 0.5 * m2 / (U[0] * U[0]);
}

/* Limiter step 4: t in [0,1] with e((1-t) Ubar + t W) = eps.  Along
 * U(t) = Ubar + t (W - Ubar), rho(t) e(U(t)) - eps rho(t)^2 =
 * rho E - |m|^2/2 - eps rho^2 is the quadratic A t^2 + B t + C with C >= 0 and
 * a negative value at t = 1; its root in [0,1] is 2C / (-B + sqrt(B^2 - 4AC)). */
static double pp_root(int ncomp, double eps, const double *Ub, const double *W)
{
    int ie = ncomp - 1;
    double D[4];
    for (int k = 0; k < ncomp; ++k) D[k] = W[k] - Ub[k];
    double dm2 = 0.0, mdm = 0.0, m2 = 0.0;
    for (int k = 1; k < ie; ++k) {
        dm2 += D[k] * D[k];
        mdm += Ub[k] * D[k];
        m2 += Ub[k] * Ub[k];
    }
    double A = D[0] * D[ie] - 0.5 * dm2 - eps * D[0] * D[0];
    double B = Ub[0] * D[ie] + Ub[ie] * D[0] - mdm - 2.0 * eps * Ub[0] * D[0];
    double C = Ub[0] * Ub[ie] - 0.5 * m2 - eps * Ub[0] * Ub[0];
    if (C <= 0.0) return 0.0;
    double disc = B * B - 4.0 * A * C;
    if (disc < 0.0) disc = 0.0;
    double t = 2.0 * C / (-B + sqrt(disc));
    if (!(t >= 0.0)) t = 0.0;
    if (t > 1.0) t = 1.0;
    return t;
}

/* Positivity-preserving limiter of one cell (Sec 2.4, steps 1-4).
 * Um = U-_{j+1/2}, Up = U+_{j-1/2}, modified in place.  Returns 1 if the
 * limiter changed anything.  Readings: rho_min is the minimum of the three
 * densities and theta1 = 1 whenever rho_min >= eps_rho; eps_e is the
 * internal-energy threshold (min(cap, min e(Ubar)) over the grid). */
static int pp_limit(int ncomp, double w1, double eps_rho, double eps_e, const double *Ub,
                    double *Um, double *Up)
{
    int active = 0;
    /* step 2 */
    double rmid = (Ub[0] - w1 * Up[0] - w1 * Um[0]) / (1.0 - 2.0 * w1);
    double rmin = fmin(fmin(Um[0], Up[0]), rmid);
    double th1 = 1.0;
    if (rmin < eps_rho) th1 = fmin((Ub[0] - eps_rho) / (Ub[0] - rmin), 1.0);
    /* step 3 */
    if (th1 < 1.0) {
        Um[0] = th1 * (Um[0] - Ub[0]) + Ub[0];
        Up[0] = th1 * (Up[0] - Ub[0]) + Ub[0];
        active = 1;
    }
    double W[3][4];
    for (int k = 0; k < ncomp; ++k) {
        W[0][k] = Um[k];
        W[1][k] = Up[k];
        W[2][k] = (Ub[k] - w1 * Up[k] - w1 * Um[k]) / (1.0 - 2.0 * w1);
    }
    /* step 4 */
    double th2 = 1.0;
    for (int al = 0; al < 3; ++al) {
        if (!(W[al][0] > 0.0) || spec_e(ncomp, W[al]) < eps_e) {
            double t = pp_root(ncomp, eps_e, Ub, W[al]);
            if (t < th2) th2 = t;
        }
    }
    if (th2 < 1.0) {
        for (int k = 0; k < ncomp; ++k) {
            Um[k] = th2 * (Um[k] - Ub[k]) + Ub[k];
            Up[k] = th2 * (Up[k] - Ub[k]) + Ub[k];
        }
        active = 1;
    }
    return active;
}

/* Exported single-cell limiter for unit tests (in-place on Um, Up). */
int orc_limit_cell(int ncomp, double w1, double eps_rho, double eps_e, const double *Ub,
                   double *Um, double *Up)
{
    return pp_limit(ncomp, w1, eps_rho, eps_e, Ub, Um, Up);
}

/* Limiter step 1 over a set of cells ([ncomp][ncell]): eps_rho = min(cap, min rho);
 * reading: eps_e = min(cap, min e(Ubar)). */
void orc_eps(long ncell, int ncomp, const double *U, double cap, double *eps_rho, double *eps_e)
{
    double er = cap, ee = cap, cell[4];
    for (long i = 0; i < ncell; ++i) {
        for (int k = 0; k < ncomp; ++k) cell[k] = U[(long)k * ncell + i];
        if (cell[0] < er) er = cell[0];
        double e = spec_e(ncomp, cell);
        if (e < ee) ee = e;
    }
    *eps_rho = er;
    *eps_e = ee;
}

/* ------------------------------------------------------------ Sec 2.1, 2.4
 * Spatial operator of one line: L_i = -(F_{i+1/2} - F_{i-1/2}) / h, with the
 * compact-WENO reconstruction, the limiter and the HLLC flux.  u and L are
 * [ncomp][n]; nrm is the component index of the normal momentum.
 * Returns the number of limited cells, or a negative error code. */
long orc_line_op(int n, int ncomp, int nrm, const double *u, int bc_lo, int bc_hi, double h,
                 const orc_params *P, double eps_rho, double eps_e, double *L, orc_line_dbg *dbg,
                 double *smax)
{
    int cyclic = (bc_lo == 0);
    int ne = n + 2 * NG;
    size_t need = (size_t)ncomp * (size_t)ne + 4u * (size_t)ncomp * (size_t)n +
                  (size_t)ncomp * (size_t)(n + 1) + 9u * (size_t)n;
    double *mem = (double *)malloc(sizeof(double) * need);
    if (!mem) return -2;
    double *ue = mem;                            /* [ncomp][ne] */
    double *um = ue + (size_t)ncomp * ne;        /* [ncomp][n] */
    double *up = um + (size_t)ncomp * n;
    double *uml = up + (size_t)ncomp * n;
    double *upl = uml + (size_t)ncomp * n;
    double *F = upl + (size_t)ncomp * n;         /* [ncomp][n+1] */
    double *work = F + (size_t)ncomp * (n + 1);  /* 9n */

    /* ghost fill (reading: transmissive = copy of the edge cell, reflective =
     * mirror image with the normal momentum negated; periodic = wrap) */
    for (int k = 0; k < ncomp; ++k) {
        double *e = ue + (size_t)k * ne;
        const double *x = u + (size_t)k * n;
        for (int i = 0; i < n; ++i) e[i + NG] = x[i];
        for (int g = 1; g <= NG; ++g) {
            double lo, hi;
            if (bc_lo == 0) lo = x[((-g) % n + n) % n];
            else if (bc_lo == 1) lo = x[0];
            else lo = (k == nrm ? -1.0 : 1.0) * x[g - 1 < n ? g - 1 : n - 1];
            if (bc_hi == 0) hi = x[(n - 1 + g) % n];
            else if (bc_hi == 1) hi = x[n - 1];
            else hi = (k == nrm ? -1.0 : 1.0) * x[n - g >= 0 ? n - g : 0];
            e[NG - g] = lo;
            e[n - 1 + NG + g] = hi;
        }
    }

    if (P->recon == 3 && !P->first_order) {
        /* characteristic-wise (Sec. 2.3): all components at once, with the
         * eigenvectors of the flux Jacobian along the line */
        int s = (ncomp == 3 || ncomp == 4) ? recon_char(ncomp, nrm, n, cyclic, ue, P, um, up) : -3;
        if (s) { free(mem); return -10 + s; }
    } else
    /* reconstruction, component by component (conservative variables) */
    for (int k = 0; k < ncomp; ++k) {
        double *mk = um + (size_t)k * n, *pk = up + (size_t)k * n;
        if (P->first_order) {
            for (int i = 0; i < n; ++i) mk[i] = pk[i] = u[(size_t)k * n + i];
        } else {
            int s = recon_scalar(n, cyclic, ue + (size_t)k * ne, P, mk, pk, work);
            if (s) { free(mem); return -10 + s; }
        }
    }

    /* limiter, cell by cell */
    long nlim = 0;
    for (int i = 0; i < n; ++i) {
        double Ub[4], Um[4], Up[4];
        for (int k = 0; k < ncomp; ++k) {
            Ub[k] = u[(size_t)k * n + i];
            Um[k] = um[(size_t)k * n + i];
            Up[k] = up[(size_t)k * n + i];
        }
        if (P->limiter) nlim += pp_limit(ncomp, P->gl_w1, eps_rho, eps_e, Ub, Um, Up);
        for (int k = 0; k < ncomp; ++k) {
            uml[(size_t)k * n + i] = Um[k];
            upl[(size_t)k * n + i] = Up[k];
        }
        if (smax) {
            /* reading of (CFL-CD): the sup-norm of |u|+a runs over the cell
             * averages and the limited interface states */
            if (*smax == *smax) {
                max_into(smax, wave_speed(P->gamma, ncomp, nrm, Ub));
                max_into(smax, wave_speed(P->gamma, ncomp, nrm, Um));
                max_into(smax, wave_speed(P->gamma, ncomp, nrm, Up));
            }
        }
    }

    /* fluxes at faces 0..n; face f lies between cells f-1 and f */
    for (int f = 0; f <= n; ++f) {
        double Ul[4], Ur[4], Ff[4];
        if (f > 0 && f < n) {
            for (int k = 0; k < ncomp; ++k) {
                Ul[k] = uml[(size_t)k * n + f - 1];
                Ur[k] = upl[(size_t)k * n + f];
            }
        } else if (cyclic) {
            for (int k = 0; k < ncomp; ++k) {
                Ul[k] = uml[(size_t)k * n + n - 1];
                Ur[k] = upl[(size_t)k * n + 0];
            }
        } else if (f == 0) {
            /* reading: image state outside the left boundary */
            for (int k = 0; k < ncomp; ++k) {
                Ur[k] = upl[(size_t)k * n + 0];
                Ul[k] = (bc_lo == 2 && k == nrm) ? -Ur[k] : Ur[k];
            }
        } else {
            for (int k = 0; k < ncomp; ++k) {
                Ul[k] = uml[(size_t)k * n + n - 1];
                Ur[k] = (bc_hi == 2 && k == nrm) ? -Ul[k] : Ul[k];
            }
        }
        if (P->flux == 1)
            lf(P->gamma, ncomp, nrm, Ul, Ur, Ff);
        else
            hllc(P->gamma, ncomp, nrm, Ul, Ur, Ff);
        for (int k = 0; k < ncomp; ++k) F[(size_t)k * (n + 1) + f] = Ff[k];
    }

    /* eq. (1DEulerFV-b) */
    for (int k = 0; k < ncomp; ++k)
        for (int i = 0; i < n; ++i)
            L[(size_t)k * n + i] = -(F[(size_t)k * (n + 1) + i + 1] - F[(size_t)k * (n + 1) + i]) / h;

    if (dbg) {
        size_t cn = (size_t)ncomp * n;
        if (dbg->um) memcpy(dbg->um, um, sizeof(double) * cn);
        if (dbg->up) memcpy(dbg->up, up, sizeof(double) * cn);
        if (dbg->um_l) memcpy(dbg->um_l, uml, sizeof(double) * cn);
        if (dbg->up_l) memcpy(dbg->up_l, upl, sizeof(double) * cn);
        if (dbg->flux) memcpy(dbg->flux, F, sizeof(double) * (size_t)ncomp * (n + 1));
    }
    free(mem);
    return nlim;
}

/* Scalar reconstruction hook for tests: ue[0..n+5] ghost-extended averages
 * (cells -3..n+2), cyclic = 1 for a periodic line.  Returns 0 on success. */
int orc_recon_scalar(int n, int cyclic, const double *ue, const orc_params *P, double *um, double *up)
{
    double *work = (double *)malloc(sizeof(double) * 9u * (size_t)n);
    if (!work) return -2;
    int s = recon_scalar(n, cyclic, ue, P, um, up, work);
    free(work);
    return s;
}

/* ------------------------------------------------------------------- 1D */
long orc_rhs_1d(int n, const double *U, int bc_lo, int bc_hi, double h, const orc_params *P,
                double *L)
{
    double er, ee;
    orc_eps(n, 3, U, P->eps_cap, &er, &ee);
    return orc_line_op(n, 3, 1, U, bc_lo, bc_hi, h, P, er, ee, L, NULL, NULL);
}

/* eq. (RK3): stage s (1, 2, 3) of the SSP Runge-Kutta method, written as printed. */
static void rk3_combine(long m, int stage, double dt, const double *U0, const double *Us,
                        const double *L, double *Uo)
{
    for (long i = 0; i < m; ++i) {
        if (stage == 1) Uo[i] = U0[i] + dt * L[i];
        else if (stage == 2) Uo[i] = 0.75 * U0[i] + 0.25 * Us[i] + 0.25 * dt * L[i];
        else Uo[i] = U0[i] / 3.0 + 2.0 / 3.0 * Us[i] + 2.0 / 3.0 * dt * L[i];
    }
}

void orc_rk3_combine(long m, int stage, double dt, const double *U0, const double *Us,
                     const double *L, double *Uo)
{
    rk3_combine(m, stage, dt, U0, Us, L, Uo);
}

long orc_stage_1d(int n, const double *U0, const double *Us, double *Uo, int stage, double dt,
                  int bc_lo, int bc_hi, double h, const orc_params *P)
{
    double *L = (double *)malloc(sizeof(double) * 3u * (size_t)n);
    if (!L) return -2;
    long r = orc_rhs_1d(n, Us, bc_lo, bc_hi, h, P, L);
    if (r >= 0) rk3_combine(3L * n, stage, dt, U0, Us, L, Uo);
    free(L);
    return r;
}

/* max over cells of |u| + a of the cell averages. */
double orc_max_speed_1d(int n, const double *U, double gamma)
{
    double s = 0.0, cell[3];
    for (int i = 0; i < n && s == s; ++i) {
        cell[0] = U[i]; cell[1] = U[n + i]; cell[2] = U[2 * n + i];
        max_into(&s, wave_speed(gamma, 3, 1, cell));
    }
    return s;
}

/* Spatial operator of a stage input together with the sup-norm of |u|+a
 * over the cell averages and the limited interface states (the norm of
 * condition (CFL-CD) under the time-step rule ORC_DT_PP below). */
long orc_rhs_speed_1d(int n, const double *U, int bc_lo, int bc_hi, double h, const orc_params *P,
                      double *L, double *smax)
{
    double er, ee;
    orc_eps(n, 3, U, P->eps_cap, &er, &ee);
    *smax = 0.0;
    return orc_line_op(n, 3, 1, U, bc_lo, bc_hi, h, P, er, ee, L, NULL, smax);
}

/* Time-step rules: 0 -> dt = cfl h / S        (condition (CFL-CD));
 *                  1 -> dt = cfl h^(5/3) / S  (Example 3.1, Table 1),
 * with S = max(|u|+a) over the cell averages at the start of the step;
 *                  2 -> dt = cfl h / S with S over the cell averages AND the
 * limited interface states of the step's input (ORC_DT_PP).  The theorem of
 * Sec. 2.4 writes the scheme as first-order HLLC steps of the interface
 * states (the H_1, H_M of its proof), so its condition (CFL-CD) bounds
 * |u|+a of those states, not only of the averages.  Under rule 2 the inputs
 * of stages 2 and 3 are checked against the same bound with the step's dt:
 * a stage whose input has dt S_s / h > w^_1 is counted (out[5]).
 * In all rules the last step is shortened to land on t_end. */
#define ORC_DT_PP 2
#define ORC_DT_RESTART 3
#define ORC_MAX_HALVINGS 60
static double dt_rule_1d(int rule, double cfl, double h, double smax)
{
    return rule == 1 ? cfl * pow(h, 5.0 / 3.0) / smax : cfl * h / smax;
}

/* 1 if every cell of [3][n] is finite with rho > 0 and p > 0 (the set G). */
static int in_G_1d(int n, const double *U, double g)
{
    for (int i = 0; i < n; ++i) {
        double r = U[i], m = U[n + i], E = U[2 * n + i];
        if (!(r > 0.0) || !((g - 1.0) * (E - 0.5 * m * m / r) > 0.0)) return 0;
    }
    return 1;
}

/* The same for a 2D state [4][nc] (nc cells). */
static int in_G_2d(long nc, const double *U, double g)
{
    for (long i = 0; i < nc; ++i) {
        double r = U[i], mx = U[nc + i], my = U[2 * nc + i], E = U[3 * nc + i];
        if (!(r > 0.0) || !((g - 1.0) * (E - 0.5 * (mx * mx + my * my) / r) > 0.0)) return 0;
    }
    return 1;
}

/* Advance U ([3][n], in place) to t_end (or max_steps).  out[0] = t reached,
 * out[1] = steps, out[2] = total limited cells, out[3] = min rho, out[4] = min p
 * over all step outputs, out[5] = stages whose input broke (CFL-CD) under the
 * step's dt (rule 2 only), out[6] = steps redone with half the dt (rule 3),
 * out[7] = stage outputs with a cell outside G (rho <= 0, p <= 0 or not
 * finite; under rule 3 only those of the attempts kept).
 * Returns 0 or a negative code (-4: no valid dt). */
int orc_run_1d(int n, double *U, int bc_lo, int bc_hi, double h, const orc_params *P,
               double t_end, double cfl, int rule, long max_steps, double *out)
{
    size_t m = 3u * (size_t)n;
    double *U1 = (double *)malloc(sizeof(double) * m), *U2 = (double *)malloc(sizeof(double) * m);
    double *L = (double *)malloc(sizeof(double) * m);
    if (!U1 || !U2 || !L) { free(U1); free(U2); free(L); return -2; }
    double t = 0.0, minr = INFINITY, minp = INFINITY;
    long steps = 0, lim = 0, viol = 0, restarts = 0, outG = 0;
    int rc = 0;
    while (t < t_end && steps < max_steps) {
        long r1, r2, r3;
        double dt;
        if (rule == ORC_DT_PP) {
            double S;
            r1 = orc_rhs_speed_1d(n, U, bc_lo, bc_hi, h, P, L, &S);
            if (r1 < 0) { rc = (int)r1; break; }
            dt = cfl * h / S;
            if (!(dt > 0.0) || dt == INFINITY) { rc = -4; break; }
            if (t + dt > t_end) dt = t_end - t;
            rk3_combine((long)m, 1, dt, U, U, L, U1);
            outG += !in_G_1d(n, U1, P->gamma);
            r2 = orc_rhs_speed_1d(n, U1, bc_lo, bc_hi, h, P, L, &S);
            if (r2 >= 0) {
                if (dt * S > P->gl_w1 * h) ++viol;
                rk3_combine((long)m, 2, dt, U, U1, L, U2);
                outG += !in_G_1d(n, U2, P->gamma);
                r3 = orc_rhs_speed_1d(n, U2, bc_lo, bc_hi, h, P, L, &S);
                if (r3 >= 0) {
                    if (dt * S > P->gl_w1 * h) ++viol;
                    rk3_combine((long)m, 3, dt, U, U2, L, U1);
                    outG += !in_G_1d(n, U1, P->gamma);
                }
            } else {
                r3 = r2;
            }
        } else {
            dt = dt_rule_1d(rule, cfl, h, orc_max_speed_1d(n, U, P->gamma));
            if (!(dt > 0.0) || dt == INFINITY) { rc = -4; break; }
            if (t + dt > t_end) dt = t_end - t;
            for (int halvings = 0;; ++halvings) {
                long bad = 0;   /* stage outputs of this attempt outside G */
                r1 = orc_stage_1d(n, U, U, U1, 1, dt, bc_lo, bc_hi, h, P);
                bad += r1 >= 0 && !in_G_1d(n, U1, P->gamma);
                r2 = r1 >= 0 ? orc_stage_1d(n, U, U1, U2, 2, dt, bc_lo, bc_hi, h, P) : r1;
                bad += r2 >= 0 && !in_G_1d(n, U2, P->gamma);
                r3 = r2 >= 0 ? orc_stage_1d(n, U, U2, U1, 3, dt, bc_lo, bc_hi, h, P) : r2;
                bad += r3 >= 0 && !in_G_1d(n, U1, P->gamma);
                if (rule != ORC_DT_RESTART || bad == 0 || r3 < 0) {
                    outG += bad;
                    break;
                }
                /* no further attempt after ORC_MAX_HALVINGS halvings, nor once
                 * half the step no longer moves t in FP64 (a stall) */
                if (halvings == ORC_MAX_HALVINGS || t + 0.5 * dt == t) { r3 = -4; break; }
                dt *= 0.5;   /* redo the step from U^n with half the step */
                ++restarts;
            }
        }
        if (r3 < 0) { rc = (int)r3; break; }
        lim += r1 + r2 + r3;
        memcpy(U, U1, sizeof(double) * m);
        for (int i = 0; i < n; ++i) {
            double r = U[i], u = U[n + i] / r;
            double p = (P->gamma - 1.0) * (U[2 * n + i] - 0.5 * r * u * u);
            if (!(r >= minr)) minr = r;
            if (!(p >= minp)) minp = p;
        }
        t += dt;
        ++steps;
    }
    out[0] = t; out[1] = (double)steps; out[2] = (double)lim; out[3] = minr; out[4] = minp;
    out[5] = (double)viol;
    out[6] = (double)restarts;
    out[7] = (double)outG;
    free(U1); free(U2); free(L);
    return rc;
}

/* ------------------------------------------------------- 2D, Gauss nodes
 * Reading (the paper leaves genuinely multi-dimensional schemes to future
 * work, Sec. 4): a 2D finite-volume operator whose face fluxes are averages
 * over the face by three-point Gauss-Legendre quadrature.
 *  1. Along each x-line the compact reconstruction of Sec. 2.2 turns the
 *     cell averages into face values that are averages over the cell's
 *     y-extent (taken before the limiter);
 *  2. across the lines, at every x-face and side, the quartic whose averages
 *     over the five cells j-2..j+2 equal those face values gives the values
 *     at the face's three Gauss nodes (a linear fifth-order step; no WENO
 *     weights across the lines);
 *  3. per cell, the limiter steps of Sec. 2.4 act on its six node values
 *     (three on each x-face) against the cell average, with the middle state
 *     from Ubar = w1 sum_k g_k (U-_k + U+_k) + (1 - 2 w1) U_mid (g_k the
 *     Gauss weights), the 2D form of the decomposition behind the theorem;
 *  4. each face flux is the g_k-weighted sum of the numerical flux at its
 *     nodes, and L_x = -(F_{i+1/2} - F_{i-1/2}) / dx.
 * The y-direction is the same with x and y exchanged; L = L_x + L_y.
 * Ghost lines across the lines follow the ghost-cell reading: periodic wrap,
 * transmissive copy of the edge line, reflective mirror with the transverse
 * momentum negated. */

static const double GL_W[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

/* Values at the Gauss nodes -sqrt(15)/10, 0, sqrt(15)/10 (in cell widths
 * from the centre of cell 2) of the quartic whose averages over cells 0..4
 * (cell m spans [m - 2.5, m - 1.5]) are v[0..4].  The quartic's monomial
 * coefficients come from the 5x5 system of monomial cell averages. */
int orc_gauss_nodes(const double *v, double *out)
{
    double M[25], a[5];
    for (int m = 0; m < 5; ++m)
        for (int p = 0; p < 5; ++p) {
            double hi = (m - 2) + 0.5, lo = (m - 2) - 0.5;
            M[m * 5 + p] = (pow(hi, p + 1) - pow(lo, p + 1)) / (p + 1);
        }
    int s = orc_dense_solve(5, M, v, a);
    if (s) return s;
    double xi[3] = {-sqrt(15.0) / 10.0, 0.0, sqrt(15.0) / 10.0};
    for (int k = 0; k < 3; ++k) {
        double q = 0.0, x = 1.0;
        for (int p = 0; p < 5; ++p) {
            q += a[p] * x;
            x *= xi[k];
        }
        out[k] = q;
    }
    return 0;
}

/* middle state of the decomposition in step 3 above */
static void node_mid(int ncomp, double w1, const double *Ub, double Nm[3][4], double Np[3][4],
                     double *mid)
{
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += GL_W[k] * (Nm[k][c] + Np[k][c]);
        mid[c] = (Ub[c] - w1 * s) / (1.0 - 2.0 * w1);
    }
}

/* Limiter steps 2-4 of Sec. 2.4 on the node states of one cell: Nm[k] the
 * nodes of its right face (U-), Np[k] those of its left face (U+), modified
 * in place.  Returns 1 if anything changed. */
static int pp_limit_nodes(int ncomp, double w1, double eps_rho, double eps_e, const double *Ub,
                          double Nm[3][4], double Np[3][4])
{
    int active = 0;
    double mid[4];
    /* step 2: theta1 from the smallest density of the seven states */
    node_mid(ncomp, w1, Ub, Nm, Np, mid);
    double rmin = mid[0];
    for (int k = 0; k < 3; ++k) rmin = fmin(rmin, fmin(Nm[k][0], Np[k][0]));
    double th1 = 1.0;
    if (rmin < eps_rho) th1 = fmin((Ub[0] - eps_rho) / (Ub[0] - rmin), 1.0);
    /* step 3 */
    if (th1 < 1.0) {
        for (int k = 0; k < 3; ++k) {
            Nm[k][0] = th1 * (Nm[k][0] - Ub[0]) + Ub[0];
            Np[k][0] = th1 * (Np[k][0] - Ub[0]) + Ub[0];
        }
        active = 1;
    }
    /* step 4: theta2 over the six nodes and the new middle state */
    node_mid(ncomp, w1, Ub, Nm, Np, mid);
    double th2 = 1.0;
    for (int al = 0; al < 7; ++al) {
        const double *W = al < 3 ? Nm[al] : (al < 6 ? Np[al - 3] : mid);
        if (!(W[0] > 0.0) || spec_e(ncomp, W) < eps_e) {
            double t = pp_root(ncomp, eps_e, Ub, W);
            if (t < th2) th2 = t;
        }
    }
    if (th2 < 1.0) {
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < ncomp; ++c) {
                Nm[k][c] = th2 * (Nm[k][c] - Ub[c]) + Ub[c];
                Np[k][c] = th2 * (Np[k][c] - Ub[c]) + Ub[c];
            }
        active = 1;
    }
    return active;
}

/* Exported node limiter for unit tests: Nm, Np are [3][4] row-major (node,
 * component), modified in place. */
int orc_limit_nodes(int ncomp, double w1, double eps_rho, double eps_e, const double *Ub,
                    double *Nm, double *Np)
{
    double A[3][4], B[3][4];
    for (int k = 0; k < 3; ++k)
        for (int c = 0; c < 4; ++c) {
            A[k][c] = c < ncomp ? Nm[k * 4 + c] : 0.0;
            B[k][c] = c < ncomp ? Np[k * 4 + c] : 0.0;
        }
    int r = pp_limit_nodes(ncomp, w1, eps_rho, eps_e, Ub, A, B);
    for (int k = 0; k < 3; ++k)
        for (int c = 0; c < ncomp; ++c) {
            Nm[k * 4 + c] = A[k][c];
            Np[k * 4 + c] = B[k][c];
        }
    return r;
}

/* line index of ghost line j (j < 0 or j >= nl) across the lines; *sign is
 * -1 where the transverse momentum is negated (reflective mirror) */
static int ghost_line(int j, int nl, int lo, int hi, int *sign)
{
    *sign = 1;
    if (j >= 0 && j < nl) return j;
    if (lo == 0) return ((j % nl) + nl) % nl;
    if (j < 0) {
        if (lo == 1) return 0;
        *sign = -1;
        return -1 - j < nl ? -1 - j : nl - 1;
    }
    if (hi == 1) return nl - 1;
    *sign = -1;
    return 2 * nl - 1 - j >= 0 ? 2 * nl - 1 - j : 0;
}

/* One direction of the Gauss-node operator: u and L are [4][nl][n] (nl lines
 * of n cells); nrm / tnrm index the normal / transverse momentum; bc_lo,
 * bc_hi close the lines, tb_lo, tb_hi the set of lines.  Returns the number
 * of limited cells or a negative code; smax (may be NULL) receives the
 * sup-norm of |u_n| + a over the averages and the limited node states. */
static long gauss_dir(int n, int nl, const double *u, int nrm, int tnrm, int bc_lo, int bc_hi,
                      int tb_lo, int tb_hi, double h, const orc_params *P, double er, double ee,
                      double *L, double *smax)
{
    size_t cs = (size_t)n * (size_t)nl;
    double *Wm = (double *)malloc(sizeof(double) * 4u * cs);   /* [4][nl][n] U-_{i+1/2} */
    double *Wp = (double *)malloc(sizeof(double) * 4u * cs);   /* [4][nl][n] U+_{i-1/2} */
    double *Nm = (double *)malloc(sizeof(double) * 12u * cs);  /* [nl][n][3][4] limited */
    double *Np = (double *)malloc(sizeof(double) * 12u * cs);
    if (!Wm || !Wp || !Nm || !Np) { free(Wm); free(Wp); free(Nm); free(Np); return -2; }
    int err = 0;
    long nlim = 0;
    double sm = 0.0;
    int cyclic = bc_lo == 0;
    /* step 1: face averages of every line */
#pragma omp parallel
    {
        double *line = (double *)malloc(sizeof(double) * 4u * (size_t)n);
        double *lo = (double *)malloc(sizeof(double) * 4u * (size_t)n);
        double *um = (double *)malloc(sizeof(double) * 4u * (size_t)n);
        double *up = (double *)malloc(sizeof(double) * 4u * (size_t)n);
#pragma omp for schedule(static)
        for (int l = 0; l < nl; ++l) {
            for (int k = 0; k < 4; ++k)
                for (int i = 0; i < n; ++i) line[(size_t)k * n + i] = u[k * cs + (size_t)l * n + i];
            orc_line_dbg dbg = {um, up, NULL, NULL, NULL};
            long r = orc_line_op(n, 4, nrm, line, bc_lo, bc_hi, h, P, er, ee, lo, &dbg, NULL);
            if (r < 0) err = (int)r;
            for (int k = 0; k < 4; ++k)
                for (int i = 0; i < n; ++i) {
                    Wm[k * cs + (size_t)l * n + i] = um[(size_t)k * n + i];
                    Wp[k * cs + (size_t)l * n + i] = up[(size_t)k * n + i];
                }
        }
        free(line); free(lo); free(um); free(up);
    }
    if (err) { free(Wm); free(Wp); free(Nm); free(Np); return err; }
    /* steps 2 and 3: node values across the lines, limiter per cell */
#pragma omp parallel for schedule(static) reduction(+ : nlim) reduction(max : sm)
    for (int l = 0; l < nl; ++l) {
        for (int i = 0; i < n; ++i) {
            double A[3][4], B[3][4], Ub[4], v[5], q[3];
            for (int k = 0; k < 4; ++k) {
                Ub[k] = u[k * cs + (size_t)l * n + i];
                for (int side = 0; side < 2; ++side) {
                    const double *W = side == 0 ? Wm : Wp;
                    for (int m = 0; m < 5; ++m) {
                        int sg;
                        int j = ghost_line(l + m - 2, nl, tb_lo, tb_hi, &sg);
                        v[m] = (k == tnrm ? sg : 1) * W[k * cs + (size_t)j * n + i];
                    }
                    orc_gauss_nodes(v, q);
                    for (int g = 0; g < 3; ++g) (side == 0 ? A : B)[g][k] = q[g];
                }
            }
            if (P->limiter) nlim += pp_limit_nodes(4, P->gl_w1, er, ee, Ub, A, B);
            double *dm = Nm + ((size_t)l * n + i) * 12u, *dp = Np + ((size_t)l * n + i) * 12u;
            for (int g = 0; g < 3; ++g)
                for (int k = 0; k < 4; ++k) {
                    dm[g * 4 + k] = A[g][k];
                    dp[g * 4 + k] = B[g][k];
                }
            if (smax) {
                double s = wave_speed(P->gamma, 4, nrm, Ub);
                for (int g = 0; g < 3; ++g) {
                    s = fmax(s, wave_speed(P->gamma, 4, nrm, A[g]));
                    s = fmax(s, wave_speed(P->gamma, 4, nrm, B[g]));
                }
                if (s != s) s = INFINITY;
                if (s > sm) sm = s;
            }
        }
    }
    /* step 4: Gauss sums of the node fluxes, flux differences */
#pragma omp parallel
    {
        double *F = (double *)malloc(sizeof(double) * 4u * (size_t)(n + 1));
#pragma omp for schedule(static)
        for (int l = 0; l < nl; ++l) {
            for (int f = 0; f <= n; ++f) {
                double Fs[4] = {0.0, 0.0, 0.0, 0.0};
                for (int g = 0; g < 3; ++g) {
                    double Ul[4], Ur[4], Ff[4];
                    for (int k = 0; k < 4; ++k) {
                        if (f > 0 && f < n) {
                            Ul[k] = Nm[((size_t)l * n + f - 1) * 12u + g * 4 + k];
                            Ur[k] = Np[((size_t)l * n + f) * 12u + g * 4 + k];
                        } else if (cyclic) {
                            Ul[k] = Nm[((size_t)l * n + n - 1) * 12u + g * 4 + k];
                            Ur[k] = Np[((size_t)l * n) * 12u + g * 4 + k];
                        } else if (f == 0) {
                            Ur[k] = Np[((size_t)l * n) * 12u + g * 4 + k];
                            Ul[k] = (bc_lo == 2 && k == nrm) ? -Ur[k] : Ur[k];
                        } else {
                            Ul[k] = Nm[((size_t)l * n + n - 1) * 12u + g * 4 + k];
                            Ur[k] = (bc_hi == 2 && k == nrm) ? -Ul[k] : Ul[k];
                        }
                    }
                    if (P->flux == 1)
                        lf(P->gamma, 4, nrm, Ul, Ur, Ff);
                    else
                        hllc(P->gamma, 4, nrm, Ul, Ur, Ff);
                    for (int k = 0; k < 4; ++k) Fs[k] += GL_W[g] * Ff[k];
                }
                for (int k = 0; k < 4; ++k) F[(size_t)k * (n + 1) + f] = Fs[k];
            }
            for (int k = 0; k < 4; ++k)
                for (int i = 0; i < n; ++i)
                    L[k * cs + (size_t)l * n + i] =
                        -(F[(size_t)k * (n + 1) + i + 1] - F[(size_t)k * (n + 1) + i]) / h;
        }
        free(F);
    }
    free(Wm); free(Wp); free(Nm); free(Np);
    if (smax) *smax = sm;
    return nlim;
}

/* Exported single direction for tests (the x-direction when u is [4][ny][nx]
 * with n = nx, nl = ny, nrm = 1, tnrm = 2). */
long orc_gauss_dir(int n, int nl, const double *u, int nrm, int tnrm, int bc_lo, int bc_hi,
                   int tb_lo, int tb_hi, double h, const orc_params *P, double er, double ee,
                   double *L)
{
    return gauss_dir(n, nl, u, nrm, tnrm, bc_lo, bc_hi, tb_lo, tb_hi, h, P, er, ee, L, NULL);
}

/* L = L_x + L_y of the Gauss-node operator for a [4][ny][nx] state; smax (may
 * be NULL) receives the x and y sup-norms of gauss_dir. */
long orc_rhs_2d_gauss(int nx, int ny, const double *U, const int *bc, double dx, double dy,
                      const orc_params *P, double *L, double *smax)
{
    long ncell = (long)nx * ny;
    double er, ee;
    orc_eps(ncell, 4, U, P->eps_cap, &er, &ee);
    double *Ut = (double *)malloc(sizeof(double) * 4u * (size_t)ncell);
    double *Lt = (double *)malloc(sizeof(double) * 4u * (size_t)ncell);
    if (!Ut || !Lt) { free(Ut); free(Lt); return -2; }
    double sx = 0.0, sy = 0.0;
    long r1 = gauss_dir(nx, ny, U, 1, 2, bc[0], bc[1], bc[2], bc[3], dx, P, er, ee, L,
                        smax ? &sx : NULL);
    for (int k = 0; k < 4; ++k)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) Ut[k * ncell + (long)x * ny + y] = U[k * ncell + (long)y * nx + x];
    long r2 = r1 < 0 ? r1
                     : gauss_dir(ny, nx, Ut, 2, 1, bc[2], bc[3], bc[0], bc[1], dy, P, er, ee, Lt,
                                 smax ? &sy : NULL);
    if (r2 >= 0)
        for (int k = 0; k < 4; ++k)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) L[k * ncell + (long)y * nx + x] += Lt[k * ncell + (long)x * ny + y];
    free(Ut);
    free(Lt);
    if (smax) { smax[0] = sx; smax[1] = sy; }
    if (r1 < 0) return r1;
    if (r2 < 0) return r2;
    return r1 + r2;
}

/* ------------------------------------------------------------------- 2D
 * Reading (the paper is one-dimensional): dimension by dimension.  Each x-line
 * (row) and y-line (column) is treated as a 1D line of 2D cell averages with
 * the normal momentum rho u (x) or rho v (y); L = L_x + L_y from the same
 * stage input, and the limiter of each direction uses the same averages. */
long orc_rhs_2d_speed(int nx, int ny, const double *U, const int *bc, double dx, double dy,
                      const orc_params *P, double *L, double *smax /* [2] or NULL */)
{
    if (P->fv == 1) return orc_rhs_2d_gauss(nx, ny, U, bc, dx, dy, P, L, smax);
    long ncell = (long)nx * ny;
    double er, ee;
    orc_eps(ncell, 4, U, P->eps_cap, &er, &ee);
    long nlim = 0;
    int err = 0;
    for (long i = 0; i < 4 * ncell; ++i) L[i] = 0.0;
    double *Lx = (double *)calloc((size_t)(4 * ncell), sizeof(double));
    if (!Lx) return -2;

    double sx = 0.0, sy = 0.0;
#pragma omp parallel reduction(+ : nlim) reduction(max : sx, sy)
    {
        int mx = nx > ny ? nx : ny;
        double *line = (double *)malloc(sizeof(double) * 4u * (size_t)mx);
        double *lo = (double *)malloc(sizeof(double) * 4u * (size_t)mx);
#pragma omp for schedule(static)
        for (int y = 0; y < ny; ++y) {
            for (int k = 0; k < 4; ++k)
                for (int x = 0; x < nx; ++x) line[(size_t)k * nx + x] = U[k * ncell + (long)y * nx + x];
            double s = 0.0;
            long r = orc_line_op(nx, 4, 1, line, bc[0], bc[1], dx, P, er, ee, lo, NULL, &s);
            if (s > sx || s != s) sx = s != s ? INFINITY : s;
            if (r < 0) err = (int)r; else nlim += r;
            for (int k = 0; k < 4; ++k)
                for (int x = 0; x < nx; ++x) Lx[k * ncell + (long)y * nx + x] = lo[(size_t)k * nx + x];
        }
#pragma omp for schedule(static)
        for (int x = 0; x < nx; ++x) {
            for (int k = 0; k < 4; ++k)
                for (int y = 0; y < ny; ++y) line[(size_t)k * ny + y] = U[k * ncell + (long)y * nx + x];
            double s = 0.0;
            long r = orc_line_op(ny, 4, 2, line, bc[2], bc[3], dy, P, er, ee, lo, NULL, &s);
            if (s > sy || s != s) sy = s != s ? INFINITY : s;
            if (r < 0) err = (int)r; else nlim += r;
            for (int k = 0; k < 4; ++k)
                for (int y = 0; y < ny; ++y) L[k * ncell + (long)y * nx + x] = lo[(size_t)k * ny + y];
        }
        free(line);
        free(lo);
    }
    for (long i = 0; i < 4 * ncell; ++i) L[i] = Lx[i] + L[i];
    free(Lx);
    if (smax) { smax[0] = sx; smax[1] = sy; }
    return err ? err : nlim;
}

long orc_rhs_2d(int nx, int ny, const double *U, const int *bc, double dx, double dy,
                const orc_params *P, double *L)
{
    return orc_rhs_2d_speed(nx, ny, U, bc, dx, dy, P, L, NULL);
}

long orc_stage_2d(int nx, int ny, const double *U0, const double *Us, double *Uo, int stage,
                  double dt, const int *bc, double dx, double dy, const orc_params *P)
{
    long m = 4L * nx * ny;
    double *L = (double *)malloc(sizeof(double) * (size_t)m);
    if (!L) return -2;
    long r = orc_rhs_2d(nx, ny, Us, bc, dx, dy, P, L);
    if (r >= 0) rk3_combine(m, stage, dt, U0, Us, L, Uo);
    free(L);
    return r;
}

/* out[0] = max(|u| + a), out[1] = max(|v| + a) over cells. */
void orc_max_speed_2d(int nx, int ny, const double *U, double gamma, double *out)
{
    long nc = (long)nx * ny;
    double sx = 0.0, sy = 0.0, cell[4];
    for (long i = 0; i < nc; ++i) {
        for (int k = 0; k < 4; ++k) cell[k] = U[k * nc + i];
        max_into(&sx, wave_speed(gamma, 4, 1, cell));
        max_into(&sy, wave_speed(gamma, 4, 2, cell));
    }
    out[0] = sx;
    out[1] = sy;
}

/* Reading: dt = cfl / (Sx/dx + Sy/dy) with Sx, Sy the sup-norms of |u|+a
 * and |v|+a: over the cell averages at the start of the step (rule 0), or
 * over the averages and the limited interface states of the x- and y-lines
 * of the step's input (rule 2, ORC_DT_PP, with the stage-2 and stage-3 inputs
 * checked against dt (Sx_s/dx + Sy_s/dy) <= w^_1, out[5]); last step clipped.
 * Rule 3 (ORC_DT_RESTART): rule 0's dt, and a step with a stage output
 * outside G is redone from U^n with half the dt, with the 1D rule's bounds
 * (out[6] = steps redone, out[7] = stage outputs outside G of the attempts
 * kept; -4 when the bounds end the run). */
int orc_run_2d_rule(int nx, int ny, double *U, const int *bc, double dx, double dy,
                    const orc_params *P, double t_end, double cfl, int rule, long max_steps,
                    double *out)
{
    size_t m = 4u * (size_t)nx * (size_t)ny;
    double *U1 = (double *)malloc(sizeof(double) * m), *U2 = (double *)malloc(sizeof(double) * m);
    double *L = (double *)malloc(sizeof(double) * m);
    if (!U1 || !U2 || !L) { free(U1); free(U2); free(L); return -2; }
    double t = 0.0, minr = INFINITY, minp = INFINITY, s[2];
    long steps = 0, lim = 0, viol = 0, restarts = 0, outG = 0;
    int rc = 0;
    while (t < t_end && steps < max_steps) {
        long r1, r2, r3;
        double dt;
        if (rule == ORC_DT_PP) {
            r1 = orc_rhs_2d_speed(nx, ny, U, bc, dx, dy, P, L, s);
            if (r1 < 0) { rc = (int)r1; break; }
            dt = cfl / (s[0] / dx + s[1] / dy);
            if (!(dt > 0.0) || dt == INFINITY) { rc = -4; break; }
            if (t + dt > t_end) dt = t_end - t;
            rk3_combine((long)m, 1, dt, U, U, L, U1);
            r2 = orc_rhs_2d_speed(nx, ny, U1, bc, dx, dy, P, L, s);
            r3 = r2;
            if (r2 >= 0) {
                if (dt * (s[0] / dx + s[1] / dy) > P->gl_w1) ++viol;
                rk3_combine((long)m, 2, dt, U, U1, L, U2);
                r3 = orc_rhs_2d_speed(nx, ny, U2, bc, dx, dy, P, L, s);
                if (r3 >= 0) {
                    if (dt * (s[0] / dx + s[1] / dy) > P->gl_w1) ++viol;
                    rk3_combine((long)m, 3, dt, U, U2, L, U1);
                }
            }
        } else {
            orc_max_speed_2d(nx, ny, U, P->gamma, s);
            dt = cfl / (s[0] / dx + s[1] / dy);
            if (!(dt > 0.0) || dt == INFINITY) { rc = -4; break; }
            if (t + dt > t_end) dt = t_end - t;
            for (int halvings = 0;; ++halvings) {
                long bad = 0;   /* stage outputs of this attempt outside G */
                r1 = orc_stage_2d(nx, ny, U, U, U1, 1, dt, bc, dx, dy, P);
                bad += r1 >= 0 && !in_G_2d(nx * (long)ny, U1, P->gamma);
                r2 = r1 >= 0 ? orc_stage_2d(nx, ny, U, U1, U2, 2, dt, bc, dx, dy, P) : r1;
                bad += r2 >= 0 && !in_G_2d(nx * (long)ny, U2, P->gamma);
                r3 = r2 >= 0 ? orc_stage_2d(nx, ny, U, U2, U1, 3, dt, bc, dx, dy, P) : r2;
                bad += r3 >= 0 && !in_G_2d(nx * (long)ny, U1, P->gamma);
                if (rule != ORC_DT_RESTART || bad == 0 || r3 < 0) {
                    outG += bad;
                    break;
                }
                /* the 1D rule's bounds: ORC_MAX_HALVINGS halvings, or a stall */
                if (halvings == ORC_MAX_HALVINGS || t + 0.5 * dt == t) { r3 = -4; break; }
                dt *= 0.5;   /* redo the step from U^n with half the step */
                ++restarts;
            }
        }
        if (r3 < 0) { rc = (int)r3; break; }
        lim += r1 + r2 + r3;
        memcpy(U, U1, sizeof(double) * m);
        long nc = (long)nx * ny;
        for (long i = 0; i < nc; ++i) {
            double r = U[i], u = U[nc + i] / r, v = U[2 * nc + i] / r;
            double p = (P->gamma - 1.0) * (U[3 * nc + i] - 0.5 * r * (u * u + v * v));
            if (!(r >= minr)) minr = r;
            if (!(p >= minp)) minp = p;
        }
        t += dt;
        ++steps;
    }
    out[0] = t; out[1] = (double)steps; out[2] = (double)lim; out[3] = minr; out[4] = minp;
    out[5] = (double)viol;
    out[6] = (double)restarts;
    out[7] = (double)outG;
    free(U1); free(U2); free(L);
    return rc;
}

int orc_run_2d(int nx, int ny, double *U, const int *bc, double dx, double dy,
               const orc_params *P, double t_end, double cfl, long max_steps, double *out)
{
    return orc_run_2d_rule(nx, ny, U, bc, dx, dy, P, t_end, cfl, 0, max_steps, out);
}

/* ------------------------------------------------------- batched 1D ensemble
 * Independent problems packed [3][sum n_i]; each advances with its own dt
 * (rule 0 or 2 of orc_run_1d) to t_end.  OpenMP over problems.  steps_out and
 * viol_out (either may be NULL) receive each problem's step count and its
 * count of stages that broke (CFL-CD) (rule 2).  Returns 0 or the first error. */
int orc_run_batch_rule(int nprob, const long *offsets, double *U, const int *bc, const double *dxs,
                       const orc_params *P, double t_end, double cfl, int rule, long total,
                       double *steps_out, double *viol_out)
{
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < nprob; ++i) {
        int n = (int)(offsets[i + 1] - offsets[i]);
        double *line = (double *)malloc(sizeof(double) * 3u * (size_t)n), out[8];
        for (int k = 0; k < 3; ++k)
            memcpy(line + (size_t)k * n, U + (size_t)k * total + offsets[i], sizeof(double) * n);
        int r = orc_run_1d(n, line, bc[2 * i], bc[2 * i + 1], dxs[i], P, t_end, cfl, rule, 1L << 40,
                           out);
        if (r) err = r;
        for (int k = 0; k < 3; ++k)
            memcpy(U + (size_t)k * total + offsets[i], line + (size_t)k * n, sizeof(double) * n);
        if (steps_out) steps_out[i] = out[1];
        if (viol_out) viol_out[i] = out[5];
        free(line);
    }
    return err;
}

int orc_run_batch(int nprob, const long *offsets, double *U, const int *bc, const double *dxs,
                  const orc_params *P, double t_end, double cfl, long total, double *steps_out)
{
    return orc_run_batch_rule(nprob, offsets, U, bc, dxs, P, t_end, cfl, 0, total, steps_out, NULL);
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
