/*
 * Test driver (CPU only): the oracle built with AddressSanitizer and
 * UndefinedBehaviorSanitizer, exercised on small problems that reach every
 * boundary kind, the shortest lines, the limiter near vacuum, all three
 * reconstructions, both fluxes, the 2D operator and the batched driver.
 * Any out-of-bounds access, leak or undefined operation aborts it.
 * Built and run by tests/test_oracle_sanitized.py.
 */
#include "../oracle/oracle.c"

#include <stdio.h>

static void riemann(int n, double *U, double rl, double ul, double pl, double rr, double ur,
                    double pr)
{
    for (int i = 0; i < n; ++i) {
        int left = i < n / 2;
        double r = left ? rl : rr, u = left ? ul : ur, p = left ? pl : pr;
        U[i] = r;
        U[n + i] = r * u;
        U[2 * n + i] = p / 0.4 + 0.5 * r * u * u;
    }
}

static orc_params params(int recon, int flux)
{
    orc_params P;
    P.gamma = 1.4;
    P.weno_eps = 1e-13;
    P.eps_cap = 1e-13;
    P.gl_w1 = 1.0 / 12.0;
    P.linear = 0;
    P.first_order = 0;
    P.limiter = 1;
    P.flux = flux;
    P.recon = recon;
    return P;
}

int main(void)
{
    static double U[3 * 4096], out[8];
    int failures = 0;
    const int sizes[] = {3, 4, 5, 7, 33, 130};
    const int bcs[][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}};
    for (int recon = 0; recon < 4; ++recon)   /* 3: characteristic-wise */
        for (int flux = 0; flux < 2; ++flux)
            for (unsigned si = 0; si < sizeof(sizes) / sizeof(sizes[0]); ++si)
                for (int b = 0; b < 4; ++b) {
                    int n = sizes[si];
                    if (bcs[b][0] == 0 && n < 5) continue; /* periodic needs 5 cells */
                    orc_params P = params(recon, flux);
                    riemann(n, U, 1.0, 0.3, 1.0, 0.125, -0.2, 0.1);
                    /* rule 0 (averages) and rule 2 (interface states) by turns */
                    int rule = ((si + b) & 1) ? 2 : 0;
                    int rc = orc_run_1d(n, U, bcs[b][0], bcs[b][1], 1.0 / n, &P, 0.05,
                                        1.0 / 12.0, rule, 20, out);
                    if (rc != 0) {
                        printf("1D run n=%d bc=%d,%d recon=%d flux=%d: rc %d\n", n, bcs[b][0],
                               bcs[b][1], recon, flux, rc);
                        ++failures;
                    }
                }
    /* near vacuum: the limiter acts (a run may stop with -4 by design) */
    {
        orc_params P = params(0, 0);
        riemann(200, U, 7.0, -1.0, 0.2, 7.0, 1.0, 0.2);
        int rc = orc_run_1d(200, U, 1, 1, 0.01, &P, 0.2, 1.0 / 12.0, 0, 200, out);
        if (rc != 0 && rc != -4) { printf("double rarefaction: rc %d\n", rc); ++failures; }
        riemann(200, U, 7.0, -1.0, 0.2, 7.0, 1.0, 0.2);
        rc = orc_run_1d(200, U, 1, 1, 0.01, &P, 0.2, 1.0 / 12.0, 2, 200, out);
        if (rc != 0) { printf("double rarefaction, rule 2: rc %d\n", rc); ++failures; }
    }
    /* 2D, every boundary kind on each side */
    {
        static double V[4 * 12 * 10];
        const int bc2[4] = {1, 2, 2, 1};
        for (int recon = 0; recon < 4; ++recon) {   /* 3: characteristic lines (4x4) */
            for (int j = 0; j < 10; ++j)
                for (int i = 0; i < 12; ++i) {
                    int c = j * 12 + i;
                    double r = (i < 6 && j < 5) ? 1.0 : 0.3, u = 0.2, v = -0.1, p = r;
                    V[c] = r;
                    V[120 + c] = r * u;
                    V[240 + c] = r * v;
                    V[360 + c] = p / 0.4 + 0.5 * r * (u * u + v * v);
                }
            orc_params P = params(recon, 0);
            int rc = orc_run_2d_rule(12, 10, V, bc2, 1.0 / 12, 1.0 / 10, &P, 0.02, 1.0 / 12.0,
                                     recon == 1 || recon == 3 ? 2 : 0, 10, out);
            if (rc != 0) { printf("2D run recon=%d: rc %d\n", recon, rc); ++failures; }
        }
    }
    /* batched driver: three problems of different lengths */
    {
        const long off[4] = {0, 7, 40, 140};
        const int bcb[6] = {1, 1, 1, 2, 2, 2};
        const double dxs[3] = {1.0 / 7, 1.0 / 33, 1.0 / 100};
        static double B[3 * 140], steps[3];
        for (int p = 0; p < 3; ++p) {
            int n = (int)(off[p + 1] - off[p]);
            double tmp[3 * 100];
            riemann(n, tmp, 1.0, 0.0, 1.0, 0.5, 0.0, 0.4);
            for (int c = 0; c < 3; ++c)
                for (int i = 0; i < n; ++i) B[c * 140 + off[p] + i] = tmp[c * n + i];
        }
        orc_params P = params(0, 0);
        int rc = orc_run_batch(3, off, B, bcb, dxs, &P, 0.01, 1.0 / 12.0, 140, steps);
        if (rc != 0) { printf("batched run: rc %d\n", rc); ++failures; }
    }
    printf("%s\n", failures ? "FAILED" : "ok");
    return failures ? 1 : 0;
}
