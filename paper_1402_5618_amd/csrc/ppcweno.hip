// MI355X (gfx950) implementation of the per-stage operator of the
// positivity-preserving fifth-order finite-volume compact-WENO scheme
// (arXiv 1402.5618) behind the C ABI of include/pp_cweno.h.
//
// Line kernel (one workgroup per grid line, or per problem of a batch):
//   phase 0  stage the line (and 3 ghost cells per side) in LDS;
//   phase 1  every (component, side) system gets a 64-lane wave (two waves
//            for lines longer than 2048): lane k chases chunk k of the rows
//            of eq. (CWENO-FV) in registers, the chunk separators form a
//            small tridiagonal system solved by parallel cyclic reduction in
//            LDS, then each lane back-substitutes its chunk.  The "+" system
//            is the "-" system of the mirrored line, so one code path serves
//            both sides and the "+" chase runs from the right end;
//   phase 2  the limiter (Sec 2.4) per cell, the HLLC flux per face (each
//            face once), the flux difference (eq. (1DEulerFV-b)) and the
//            epilogue: write L, or the RK3 stage combination of eq. (RK3).
// 2D: x-lines run on the [4][ny][nx] state, y-lines on a transposed copy
// [4][nx][ny]; a tiled combine kernel forms U_{s+1} = a Un + b (Us + dt (Lx + Ly)),
// writes it in both layouts and reduces the next stage's limiter epsilon and
// the next step's wave speeds with order-independent atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "pp_cweno.h"
#include "ppc_device.h"

using namespace ppc;

// Device scratch of the allocation-free entry point pp_cweno_step_static: the
// run scalars (first 256 bytes) and the two stage buffers of a 1D line of up
// to 4096 cells.  Every GPU holds its own copy; host code reaches it only
// through the address hipGetSymbolAddress returns on that device.
constexpr int kStaticMaxN = 4096;
constexpr int kStaticScalSlots = 32;   // doubles reserved for the scalars
static __device__ __align__(256) double scratch[kStaticScalSlots + 2 * 3 * kStaticMaxN];

namespace {

constexpr int kCH = 32;      // max rows of one chunk held in registers
constexpr int kNG = 3;       // ghost cells per side

// LDS padding: one spare double after every 2^SH, so lanes that stride by
// 2^SH doubles (one chunk of rows each) hit different banks.
template <int SH>
__host__ __device__ __forceinline__ int padn(int e) { return e + (e >> SH); }

// Device scalars of a run: limiter epsilons per stage slot, wave speeds,
// time step, time, step count, sticky status.
struct Scal {
    long long eps[3][2];   // slot s: encoded min rho, min e of a stage input
    long long spd[2];      // encoded max(|u|+a), max(|v|+a)
    double dt, t;
    long long steps;
    int active;
    unsigned status;
    unsigned stepbad;      // restart rule: status bits of the step being tried
    long long restarts;    // restart rule: steps redone with half the dt
    long long spdif[2];    // 2D interface-state rule: encoded max |u|+a, |v|+a over the
                           // averages and limited interface states of a stage input
    long long eps3[2];     // restart rule, 2D: epsilons of the stage-3 output being tried
    int redo;              // restart rule, host-driven runs: the next step is a retry
    int halvings;          //   halvings of the step being tried
};

// Steps redone with half the dt before a run gives up (restart rule).
constexpr int kMaxHalvings = 60;

struct LineArgs {
    const double* U;        // stage input
    const double* U0;       // RK base (stage mode)
    double* out;            // L (mode 0) or stage output (mode 1)
    long long cs;           // component stride
    long long ls;           // line stride (used when off == nullptr)
    const long long* off;   // batched: element offset of each problem
    const int* nline;       // batched: cells of each problem
    const double* hline;    // batched: spacing of each problem
    const int* bcline;      // batched: [2] boundary codes of each problem
    double* dtline;         // batched: dt of each problem (<= 0: inactive)
    double* tline;          // batched: time of each problem
    long long* stepline;    // batched: steps taken by each problem (stage-3 advance)
    long long steps_max;    // batched: step budget per problem
    const int* order;       // batched: processing order (longest first)
    int* counter;           // batched: persistent work counter
    int n, nlines;
    int bc_lo, bc_hi;
    int seg_max;            // max cells per phase-2 segment
    int flux;               // PP_FLUX_HLLC or PP_FLUX_LF
    double h, gamma, w1, i12, weno_eps, eps_cap, t_end, cfl;
    const long long* eps_enc;  // encoded (min rho, min e) of the whole grid, or nullptr
    const double* dt_dev;      // stage mode: dt on the device, or nullptr -> dt_val
    double dt_val;
    double rk_a, rk_b;
    int mode;               // 0: write L; 1: write the stage combination
    int stage;              // 1..3 (batched stage 3 advances dt and t)
    Scal* scal;             // single grid: active flag, status, speed reduction
    unsigned* status;
    double* dbg_um;
    double* dbg_up;
    double* dbg_flux;
    long long* spd_if;      // 2D sweeps under the interface-state rule: encoded max of
                            // |u_n|+a over the averages and limited interface states
    int dtrule;             // PP_DT_*: PP_DT_PP reduces |u|+a over the limited interface
                            // states; PP_DT_RESTART commits stage 3 only if the step stayed in G
    unsigned* badline;      // batched, restart rule: status bits of each problem's step
    int* halfline;          // batched, restart rule: halvings of each problem's current step
    double* commit;         // batched, restart rule: state the stage-3 output is copied into
    unsigned long long* restart_count;   // batched, restart rule: redone steps (all problems)
    double* chs;            // characteristic reconstruction: scratch of the block solves
    long long chs_side;     //   doubles of one side's row scratch
    long long chs_line;     //   doubles of one line's scratch (0: one line)
};

template <int NT>
__device__ __forceinline__ void block_min2(double& a, double& b, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a = fmin(a, __shfl_xor(a, o));
        b = fmin(b, __shfl_xor(b, o));
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) {
        red[2 * w] = a;
        red[2 * w + 1] = b;
    }
    __syncthreads();
    a = red[0];
    b = red[1];
    for (int i = 1; i < NT / 64; ++i) {
        a = fmin(a, red[2 * i]);
        b = fmin(b, red[2 * i + 1]);
    }
    __syncthreads();
}

template <int NT>
__device__ __forceinline__ double block_max(double a, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = a;
    __syncthreads();
    a = red[0];
    for (int i = 1; i < NT / 64; ++i) a = fmax(a, red[i]);
    __syncthreads();
    return a;
}

// Values of lane src of this system (src in [0, P)): lane shuffles when one
// wave holds the system, else an LDS round trip (all threads must call).
template <int W, int NV>
__device__ __forceinline__ void xch(double (&v)[NV], int src, double* sx, int sys, int k) {
    constexpr int LANES = 64 * W;
    if constexpr (W == 1) {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = __shfl(v[i], src);
    } else {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NV; ++i) sx[(sys * LANES + k) * 4 + i] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = sx[(sys * LANES + src) * 4 + i];
    }
}

// Parallel cyclic reduction of the separator system of one (component,
// side): row k is A R_{k-1} + B R_k + C R_{k+1} = D over P lanes (indices mod P
// when cyclic).  Returns R_k.  Arithmetic in T.
template <int W, typename T>
__device__ __forceinline__ T pcr_solve(T A, T B, T C, T D, int k, int P, bool cyclic, double* sx,
                                       int sys) {
    for (int s = 1; s < P; s <<= 1) {
        const int km = (k - s) & (P - 1), kp = (k + s) & (P - 1);
        double m[4] = {(double)A, (double)B, (double)C, (double)D};
        double p[4] = {(double)A, (double)B, (double)C, (double)D};
        xch<W, 4>(m, km, sx, sys, k);
        xch<W, 4>(p, kp, sx, sys, k);
        T Am = (T)m[0], Bm = (T)m[1], Cm = (T)m[2], Dm = (T)m[3];
        T Ap = (T)p[0], Bp = (T)p[1], Cp = (T)p[2], Dp = (T)p[3];
        if (!cyclic) {
            if (k - s < 0) { Am = T(0); Bm = T(1); Cm = T(0); Dm = T(0); }
            if (k + s >= P) { Ap = T(0); Bp = T(1); Cp = T(0); Dp = T(0); }
        }
        const T al = -A * rcp_t(Bm), bt = -C * rcp_t(Bp);
        const T nA = al * Am, nC = bt * Cp;
        const T nB = B + al * Cm + bt * Ap, nD = D + al * Dm + bt * Dp;
        A = nA; B = nB; C = nC; D = nD;
    }
    return cyclic ? D / (A + B + C) : D / B;
}

// Parallel cyclic reduction of a tridiagonal system of M <= 64 unknowns held
// one row per lane of a single wave (lane shuffles, no barriers).  Row l:
// a y_{l-1} + b y_l + c y_{l+1} = d, indices mod M when cyclic.  Returns y_l.
__device__ __forceinline__ double pcr_wave(double a, double b, double c, double d, int l, int M,
                                           bool cyclic) {
    for (int s = 1; s < M; s <<= 1) {
        const int lm = (l - s) & (M - 1), lp = (l + s) & (M - 1);
        double am = __shfl(a, lm), bm = __shfl(b, lm), cm = __shfl(c, lm), dm = __shfl(d, lm);
        double ap = __shfl(a, lp), bp = __shfl(b, lp), cp = __shfl(c, lp), dp = __shfl(d, lp);
        if (!cyclic) {
            if (l - s < 0) { am = 0.0; bm = 1.0; cm = 0.0; dm = 0.0; }
            if (l + s >= M) { ap = 0.0; bp = 1.0; cp = 0.0; dp = 0.0; }
        }
        const double al = -a * rcp_pos(bm), bt = -c * rcp_pos(bp);
        const double na = al * am, nc = bt * cp;
        const double nb = b + al * cm + bt * ap, nd = d + al * dm + bt * dp;
        a = na; b = nb; c = nc; d = nd;
    }
    return cyclic ? d / (a + b + c) : d / b;
}

// Separator systems of one component, P <= 128 unknowns each: the "-" system
// in lane order and the "+" system in mirrored order (index P-1-k for lane k).
// The rows go through LDS to one wave per system (wave 0 of the component:
// "-", wave 1: "+").  With P = 128 each lane takes an even and an odd row,
// eliminates the even unknowns (one cyclic-reduction step; the next lane's
// even row by shuffle), the 64 odd unknowns are solved by pcr_wave and the
// even ones recovered; with P <= 64 one row per lane.  Lane k receives its
// separators R (own) and L (previous in elimination order) of both systems.
// sxc: this component's [8][128] LDS slots.  All threads of the block call.
__device__ __forceinline__ void sep_solve_pair(const double (&A)[2], const double (&B)[2],
                                               const double (&C)[2], const double (&D)[2], int k,
                                               int P, bool cyclic, double* sxc, double& Rm,
                                               double& Lm, double& Rp, double& Lp) {
    __syncthreads();
    if (k < P) {
        const int ii[2] = {k, P - 1 - k};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            sxc[q * 512 + ii[q]] = A[q];
            sxc[q * 512 + 128 + ii[q]] = B[q];
            sxc[q * 512 + 256 + ii[q]] = C[q];
            sxc[q * 512 + 384 + ii[q]] = D[q];
        }
    }
    __syncthreads();
    const int q = k >> 6, l = k & 63;
    double* row = sxc + q * 512;   // rows of system q; results go to its A slots
    if (P == 128) {
        const int e = 2 * l, o = 2 * l + 1;
        const double Ae = row[e], Be = row[128 + e], Ce = row[256 + e], De = row[384 + e];
        const double Ao = row[o], Bo = row[128 + o], Co = row[256 + o], Do = row[384 + o];
        const int ln = (l + 1) & 63;
        double An = __shfl(Ae, ln), Bn = __shfl(Be, ln), Cn = __shfl(Ce, ln), Dn = __shfl(De, ln);
        if (!cyclic && l == 63) { An = 0.0; Bn = 1.0; Cn = 0.0; Dn = 0.0; }
        const double al = -Ao * rcp_pos(Be), bt = -Co * rcp_pos(Bn);
        const double y = pcr_wave(al * Ae, Bo + al * Ce + bt * An, bt * Cn, Do + al * De + bt * Dn,
                                  l, 64, cyclic);
        double ym = __shfl(y, (l - 1) & 63);
        if (!cyclic && l == 0) ym = 0.0;
        const double x = (De - Ae * ym - Ce * y) / Be;
        row[e] = x;
        row[o] = y;
    } else {
        const double a = l < P ? row[l] : 0.0, b = l < P ? row[128 + l] : 1.0;
        const double c = l < P ? row[256 + l] : 0.0, d = l < P ? row[384 + l] : 0.0;
        const double y = pcr_wave(a, b, c, d, l, P, cyclic);
        if (l < P) row[l] = y;
    }
    __syncthreads();
    Rm = sxc[k & (P - 1)];
    Lm = (!cyclic && k == 0) ? 0.0 : sxc[(k - 1) & (P - 1)];
    Rp = sxc[512 + ((P - 1 - k) & (P - 1))];
    Lp = (!cyclic && k + 1 >= P) ? 0.0 : sxc[512 + ((P - 2 - k) & (P - 1))];
}

constexpr int kCHP = 16;   // paired FP64 path: rows per lane and side

// Phase 1 of the paired FP64 path: lane k of a component holds rows
// [r0, r0 + len) of both tridiagonal systems of that component.
//  "-" system (eq. (CWENO-FV)): x_j = u-_{j+1/2}, row j couples x_{j-1}, x_j, x_{j+1}.
//  "+" system (its mirror):     y_j = u+_{j-1/2}, row j couples y_{j+1}, y_j, y_{j-1}
//  and is eliminated from the right end, within the chunk and through the
//  separator system.  The smoothness indicators of cell j serve both rows of
//  cell j; the "+" weights are the "-" weight products in mirrored order.
// On return E0[j] = x_{r0+j}, F0[j] = y_{r0+j}.  All threads of the block
// must call.  FULL: every lane holds exactly kCHP rows (n = kCHP P), so the
// row guards of the unrolled loops vanish and each pass is one basic block.
template <bool FULL>
__device__ __forceinline__ void paired_solve(const double* __restrict__ sUc, int n, int k, int P,
                                             bool cyclic, double weps, double* sxc, double* cl,
                                             int r0,
                                             int len, double (&E0)[kCHP], double (&E1)[kCHP],
                                             double (&E2)[kCHP], double (&F0)[kCHP],
                                             double (&F1)[kCHP], double (&F2)[kCHP]) {
    const double k13 = 13.0 / 12.0;
    const bool act = k < P;
    const int L = FULL ? kCHP : len;
    // cell average of cell r0 + rel (rel >= -3)
    auto vrel = [&](int rel) -> double { return sUc[padn<4>(r0 + rel + kNG)]; };
    auto vabs = [&](int m) -> double { return sUc[padn<4>(m + kNG)]; };
    // A non-periodic line is closed by the values just outside it ("-" side
    // x_{-1}, x_n at nodes -1/2, n+1/2 seen from the ghost cells; "+" side
    // y_{-1}, y_n, their mirror images).  They are formed first, parked in
    // LDS (cl[0..3]) and applied after the chunk passes, which keeps them out
    // of the unrolled loops: x_n and y_{-1} belong to the separator rows of
    // the last / first chunk, x_{-1} and y_n are the L of the first "-" /
    // last "+" chunk.
    if (act && !cyclic && k == 0) {
        cl[0] = weno5z_value(vabs(-3), vabs(-2), vabs(-1), vabs(0), vabs(1), weps);   // x_{-1}
        cl[1] = weno5z_value(vabs(1), vabs(0), vabs(-1), vabs(-2), vabs(-3), weps);   // y_{-1}
    }
    if (act && !cyclic && k == P - 1) {
        cl[2] = weno5z_value(vabs(n - 2), vabs(n - 1), vabs(n), vabs(n + 1), vabs(n + 2),
                             weps);                                                     // x_n
        cl[3] = weno5z_value(vabs(n + 2), vabs(n + 1), vabs(n), vabs(n - 1), vabs(n - 2),
                             weps);                                                     // y_n
    }
    // "-": x_j = P + Q L + S R, L = x_{r0-1}, R = x_{r1-1} (separator)
    // "+": y_j = P + Q L + S R, L = y_{r1},  R = y_{r0}   (separator)
    double ae = 0.0, be = 1.0, ce = 0.0, re = 0.0;
    double gP = 0.0, gQ = 1.0, gS = 0.0, fP = 0.0, fQ = 0.0, fS = 1.0;
    double aeP = 0.0, beP = 1.0, ceP = 0.0, reP = 0.0;
    double gPp = 0.0, gQp = 1.0, gSp = 0.0, fPp = 0.0, fQp = 0.0, fSp = 1.0;
    if (act) {
        // pass 1, ascending: indicators and both weight sets; "-" chasing;
        // the "+" weights (w0, w2) are kept for the descending pass
        double v0 = vrel(-2), v1 = vrel(-1), v2 = vrel(0), v3 = vrel(1);
        double d2m = v0 - 2.0 * v1 + v2, d2c = v1 - 2.0 * v2 + v3;
        double qm = k13 * d2m * d2m, qc = k13 * d2c * d2c;
        double cprev = 0.0, pprev = 0.0, qprev = 0.0;
#pragma unroll
        for (int j = 0; j < kCHP; ++j) {
            if (j < L) {
                const int g = r0 + j;
                const double v4 = vrel(j + 2);
                const double d2p = v2 - 2.0 * v3 + v4;
                const double qp = k13 * d2p * d2p;
                const double t0 = v0 - 4.0 * v1 + 3.0 * v2, t1 = v1 - v3;
                const double t2 = 3.0 * v2 - 4.0 * v3 + v4;
                const double b0 = qm + 0.25 * t0 * t0;
                const double b1 = qc + 0.25 * t1 * t1;
                const double b2 = qp + 0.25 * t2 * t2;
                const double tau = b2 - b0, tt = tau * tau;
                const double d0 = b0 + weps, d1 = b1 + weps, dd2 = b2 + weps;
                const double e0 = d0 * d0, e1 = d1 * d1, e2 = dd2 * dd2;
                const double G0 = (e0 + tt) * (e1 * e2);
                const double G1 = (e1 + tt) * (e0 * e2);
                const double G2 = (e2 + tt) * (e0 * e1);
                // "-" weights (0.2, 0.5, 0.3) on (G0, G1, G2); "+" on (G2, G1, G0).
                // The "-" rows are built from the unnormalised weights, times
                // 6: a row's scale cancels in its own pivot (chase, back
                // substitution and separator reduction alike), so that weight
                // sum is never divided out.  The "+" weights are normalised
                // (two of them are kept for pass 2, w1 = 1 - w0 - w2).
                const double am0 = 0.2 * G0, am1 = 0.5 * G1, am2 = 0.3 * G2;
                const double ap0 = 0.2 * G2, ap2 = 0.3 * G0;
                const double ipw = rcp_pos(ap0 + am1 + ap2);
                F0[j] = ap0 * ipw;
                F2[j] = ap2 * ipw;
                double a = 4.0 * am0 + 2.0 * am1, bb = 2.0 * am0 + 4.0 * (am1 + am2);
                double c = 2.0 * am2;
                double r = am0 * v1 + (5.0 * (am0 + am1) + am2) * v2 + (am1 + 5.0 * am2) * v3;
                if (j < L - 1) {
                    const double piv = (j == 0) ? bb : bb - a * cprev;
                    const double ip = rcp_pos(piv);
                    const double cj = c * ip;
                    const double pj = ((j == 0) ? r : r - a * pprev) * ip;
                    const double qj = ((j == 0) ? -a : -a * qprev) * ip;
                    E0[j] = cj; E1[j] = pj; E2[j] = qj;
                    cprev = cj; pprev = pj; qprev = qj;
                } else {
                    ae = a; be = bb; ce = c; re = r;
                }
                v0 = v1; v1 = v2; v2 = v3; v3 = v4;
                qm = qc; qc = qp;
            }
        }
        // "-" symbolic back substitution
        double Pn = 0.0, Qn = 0.0, Sn = 0.0;
#pragma unroll
        for (int j = kCHP - 1; j >= 0; --j) {
            if (j < L - 1) {
                const double cj = E0[j];
                double Pj, Qj, Sj;
                if (j == L - 2) {
                    Pj = E1[j]; Qj = E2[j]; Sj = -cj;
                    gP = Pj; gQ = Qj; gS = Sj;
                } else {
                    Pj = E1[j] - cj * Pn; Qj = E2[j] - cj * Qn; Sj = -cj * Sn;
                }
                E0[j] = Pj; E1[j] = Qj; E2[j] = Sj;
                Pn = Pj; Qn = Qj; Sn = Sj;
            }
        }
        if (L >= 2) { fP = E0[0]; fQ = E1[0]; fS = E2[0]; }
        // pass 2, descending: "+" rows (a couples y_{g+1}, c couples y_{g-1})
        double vr = vrel(L), vc = vrel(L - 1);   // v_{g+1}, v_g
        cprev = 0.0; pprev = 0.0; qprev = 0.0;
#pragma unroll
        for (int j = kCHP - 1; j >= 0; --j) {
            if (j < L) {
                const int g = r0 + j;
                const double vl = vrel(j - 1);
                const double w0 = F0[j], w2 = F2[j], w1 = 1.0 - w0 - w2;
                // (rows times 6, like the "-" rows)
                double a = 4.0 * w0 + 2.0 * w1, bb = 2.0 * w0 + 4.0 * (w1 + w2);
                double c = 2.0 * w2;
                double r = w0 * vr + (5.0 * (w0 + w1) + w2) * vc + (w1 + 5.0 * w2) * vl;
                if (j > 0) {
                    const bool first = (j == L - 1);
                    const double piv = first ? bb : bb - a * cprev;
                    const double ip = rcp_pos(piv);
                    const double cj = c * ip;
                    const double pj = (first ? r : r - a * pprev) * ip;
                    const double qj = (first ? -a : -a * qprev) * ip;
                    F0[j] = cj; F1[j] = pj; F2[j] = qj;
                    cprev = cj; pprev = pj; qprev = qj;
                } else {
                    aeP = a; beP = bb; ceP = c; reP = r;
                }
                vr = vc; vc = vl;
            }
        }
        // "+" symbolic back substitution, ascending from the separator
        Pn = 0.0; Qn = 0.0; Sn = 0.0;
#pragma unroll
        for (int j = 1; j < kCHP; ++j) {
            if (j < L) {
                const double cj = F0[j];
                double Pj, Qj, Sj;
                if (j == 1) {
                    Pj = F1[j]; Qj = F2[j]; Sj = -cj;
                    gPp = Pj; gQp = Qj; gSp = Sj;
                } else {
                    Pj = F1[j] - cj * Pn; Qj = F2[j] - cj * Qn; Sj = -cj * Sn;
                }
                F0[j] = Pj; F1[j] = Qj; F2[j] = Sj;
                Pn = Pj; Qn = Qj; Sn = Sj;
                if (j == L - 1) { fPp = Pj; fQp = Qj; fSp = Sj; }
            }
        }
    }
    double xlo = 0.0, yhi = 0.0;   // x_{-1} (lane 0), y_n (lane P-1)
    if (act && !cyclic && k == P - 1) {
        re -= ce * cl[2];   // row n-1 of "-": the separator of the last chunk
        ce = 0.0;
        yhi = cl[3];
    }
    if (act && !cyclic && k == 0) {
        reP -= ceP * cl[1];   // row 0 of "+": the separator of the first chunk
        ceP = 0.0;
        xlo = cl[0];
    }
    // first-unknown relations of the neighbour chunks: "-" from lane k+1,
    // "+" from lane k-1
    const int kn = (k + 1) & (P - 1), kq = (k - 1) & (P - 1);
    __syncthreads();
    sxc[k] = fP; sxc[128 + k] = fQ; sxc[256 + k] = fS;
    sxc[512 + k] = fPp; sxc[640 + k] = fQp; sxc[768 + k] = fSp;
    __syncthreads();
    double nf0 = sxc[kn], nf1 = sxc[128 + kn], nf2 = sxc[256 + kn];
    double np0 = sxc[512 + kq], np1 = sxc[640 + kq], np2 = sxc[768 + kq];
    if (!cyclic && k + 1 >= P) nf0 = nf1 = nf2 = 0.0;
    if (!cyclic && k == 0) np0 = np1 = np2 = 0.0;
    double RA[2] = {ae * gQ, aeP * gQp};
    double RB[2] = {be + ae * gS + ce * nf1, beP + aeP * gSp + ceP * np1};
    double RC[2] = {ce * nf2, ceP * np2};
    double RD[2] = {re - ae * gP - ce * nf0, reP - aeP * gPp - ceP * np0};
    if (!cyclic && k == 0) {   // the known x_{-1} moves to the right side
        RD[0] -= RA[0] * xlo;
        RA[0] = 0.0;
    }
    if (!cyclic && k == P - 1) {   // the known y_n likewise
        RD[1] -= RA[1] * yhi;
        RA[1] = 0.0;
    }
    double Rm, Lm, Rp, Lp;
    sep_solve_pair(RA, RB, RC, RD, k, P, cyclic, sxc, Rm, Lm, Rp, Lp);
    if (!cyclic && k == 0) Lm = xlo;
    if (!cyclic && k == P - 1) Lp = yhi;
    if (act) {
#pragma unroll
        for (int j = 0; j < kCHP; ++j) {
            if (j < L - 1) E0[j] = E0[j] + E1[j] * Lm + E2[j] * Rm;
            else if (j == L - 1) E0[j] = Rm;
            if (j == 0) F0[j] = Rp;
            else if (j < L) F0[j] = F0[j] + F1[j] * Lp + F2[j] * Rp;
        }
    }
}

// Chunked chasing of one tridiagonal system of eq. (CWENO-FV) (row g:
// a x_{g-1} + b x_g + c x_{g+1} = r, indices mod n when cyclic) over the
// P <= 64 W lanes of the system: lane k chases its rows [r0, r0 + len) with
// the chunk's separators kept symbolic (x_j = P_j + Q_j L + S_j R), the
// separator system goes through parallel cyclic reduction (pcr_solve), and
// each lane recovers its rows into E0.  row(j, a, b, c, r) returns row r0 + j
// and is called for j = 0, 1, ... in order (it may slide a window).  Every
// thread of the system calls this (W > 1 exchanges through block barriers).
template <int W, typename RowFn>
__device__ __forceinline__ void chunk_chase_solve(RowFn&& row, bool act, int k, int P, int len,
                                                  bool cyclic, double* sx, int sys,
                                                  double (&E0)[kCH], double (&E1)[kCH],
                                                  double (&E2)[kCH]) {
    const int knext = (k + 1) & (P - 1), kprev = (k - 1) & (P - 1);
    double ae = 0.0, be = 1.0, ce = 0.0, re = 0.0;
    double gP = 0.0, gQ = 1.0, gS = 0.0;   // x_{r1-2} = gP + gQ L + gS R
    double fP = 0.0, fQ = 0.0, fS = 1.0;   // x_{r0}   = fP + fQ L + fS R
    if (act) {
        double cprev = 0.0, pprev = 0.0, qprev = 0.0;
#pragma unroll
        for (int j = 0; j < kCH; ++j) {
            if (j < len) {
                double a, bb, c, r;
                row(j, a, bb, c, r);
                if (j < len - 1) {
                    const double piv = (j == 0) ? bb : bb - a * cprev;
                    const double ip = rcp_t(piv);
                    const double cj = c * ip;
                    const double pj = ((j == 0) ? r : r - a * pprev) * ip;
                    const double qj = ((j == 0) ? -a : -a * qprev) * ip;
                    E0[j] = cj; E1[j] = pj; E2[j] = qj;
                    cprev = cj; pprev = pj; qprev = qj;
                } else {
                    ae = a; be = bb; ce = c; re = r;
                }
            }
        }
        // symbolic back substitution: x_j = P_j + Q_j L + S_j R
        double Pn = 0.0, Qn = 0.0, Sn = 0.0;
#pragma unroll
        for (int j = kCH - 1; j >= 0; --j) {
            if (j < len - 1) {
                const double cj = E0[j];
                double Pj, Qj, Sj;
                if (j == len - 2) {
                    Pj = E1[j]; Qj = E2[j]; Sj = -cj;
                    gP = Pj; gQ = Qj; gS = Sj;
                } else {
                    Pj = E1[j] - cj * Pn; Qj = E2[j] - cj * Qn; Sj = -cj * Sn;
                }
                E0[j] = Pj; E1[j] = Qj; E2[j] = Sj;
                Pn = Pj; Qn = Qj; Sn = Sj;
            }
        }
        if (len >= 2) { fP = E0[0]; fQ = E1[0]; fS = E2[0]; }
    }
    double nf[3] = {fP, fQ, fS};
    xch<W, 3>(nf, knext, sx, sys, k);
    if (!cyclic && k + 1 >= P) nf[0] = nf[1] = nf[2] = 0.0;
    const double Rk = pcr_solve<W, double>(ae * gQ, be + ae * gS + ce * nf[1], ce * nf[2],
                                           re - ae * gP - ce * nf[0], k, P, cyclic, sx, sys);
    double lv[1] = {Rk};
    xch<W, 1>(lv, kprev, sx, sys, k);
    const double Lk = (!cyclic && k == 0) ? 0.0 : lv[0];
    if (act) {
#pragma unroll
        for (int j = 0; j < kCH; ++j) {
            if (j < len - 1) E0[j] = E0[j] + E1[j] * Lk + E2[j] * Rk;
            else if (j == len - 1) E0[j] = Rk;
        }
    }
}

// Test hook kernel: the chunked chase of one caller-given tridiagonal
// system (one workgroup of 64 W lanes).
template <int W>
__global__ void __launch_bounds__(64 * W) tridiag_debug_kernel(const double* __restrict__ a,
                                                               const double* __restrict__ b,
                                                               const double* __restrict__ c,
                                                               const double* __restrict__ r,
                                                               double* __restrict__ x, int n,
                                                               int cyclic) {
    __shared__ double sx[64 * W * 4];
    const int k = threadIdx.x;
    int P = 64 * W, lgP = W == 1 ? 6 : 7;
    while (P > n) {
        P >>= 1;
        --lgP;
    }
    const bool act = k < P;
    const int r0 = act ? (int)(((unsigned)k * (unsigned)n) >> lgP) : 0;
    const int r1 = act ? (int)(((unsigned)(k + 1) * (unsigned)n) >> lgP) : 0;
    double E0[kCH], E1[kCH], E2[kCH];
    auto row = [&](int j, double& aa, double& bb, double& cc, double& rr) {
        const int g = r0 + j;
        aa = a[g];
        bb = b[g];
        cc = c[g];
        rr = r[g];
        if (!cyclic) {
            if (g == 0) aa = 0.0;
            if (g == n - 1) cc = 0.0;
        }
    };
    chunk_chase_solve<W>(row, act, k, P, r1 - r0, cyclic != 0, sx, 0, E0, E1, E2);
    if (act) {
#pragma unroll
        for (int j = 0; j < kCH; ++j)
            if (j < r1 - r0) x[r0 + j] = E0[j];
    }
}

// ------------------------------------------------ Sec 2.3, characteristic
// Scratch of the characteristic block solves of one line: per side, per row
// j of a lane's chunk, kCharRec(NB) doubles per lane, lane-minor so a
// wave's accesses are coalesced; then the nodal values [side][NB][n].  The
// 2D sweeps give every line of a launch its own scratch.
constexpr int kCharRec(int nb) { return 2 * nb * nb + nb; }   // two blocks and a vector
constexpr int kCharRows(int n) { return (n + 63) / 64 + 1; }  // >= the rows of any lane's chunk
constexpr long long char_side_len(int nb, int n) { return (long long)kCharRows(n) * kCharRec(nb) * 64; }
constexpr long long char_line_len(int nb, int n) { return 2 * char_side_len(nb, n) + 2LL * nb * n; }

template <int NB>
__device__ __forceinline__ void shflN(const double (&v)[NB], int src, double (&o)[NB]) {
#pragma unroll
    for (int i = 0; i < NB; ++i) o[i] = __shfl(v[i], src);
}
template <int NB>
__device__ __forceinline__ void set_identity(double (&M)[NB * NB]) {
#pragma unroll
    for (int i = 0; i < NB * NB; ++i) M[i] = (i % (NB + 1) == 0) ? 1.0 : 0.0;
}

// One side of the characteristic-wise reconstruction of a line, by one wave
// (lane k): the NB x NB block tridiagonal system (1DEuler-FVC) whose row j
// sits at node j+1/2 of the line (the "+" side runs on the reversed line,
// as the scalar path does), A_j x_{j-1} + B_j x_j + C_j x_{j+1} = r_j with
// A_j = diag(a^(k)) L_j etc., L_j the left eigenvectors at the Roe average
// of cells j and j+1, a^(k)... the rows of eq. (CWENO-FV) built from the
// characteristic variables l^(k) . Ubar of the stencil.  NB = 3: a 1D line
// (rho, rho u, E); NB = 4: a line of the 2D operator whose normal momentum
// is component NRM, worked in the line's own order (rho, normal momentum,
// tangential momentum, E) so that x and y lines run the same arithmetic.
// Each lane chases its chunk of rows with the left separator kept
// symbolic, reduces its last row onto the separators, the separator system
// is solved by block parallel cyclic reduction across the wave, and each
// lane recovers its rows.  sU: the line in LDS ([NB][LP], ghosts included);
// scr: this side's row scratch; xs: the nodal values [NB][n] of this side
// (reversed order for the "+" side), components in the grid's order.
template <int NB, int NRM, int PSH>
__device__ __forceinline__ void char_side(const double* __restrict__ sU, int LP, int n, bool cyclic, bool rev,
                          int k, double gam, double weps, double* __restrict__ scr,
                          double* __restrict__ xs) {
    constexpr int BB = NB * NB;
    constexpr int REC = kCharRec(NB);
    int P = 64, lgP = 6;
    while (P > n) {
        P >>= 1;
        --lgP;
    }
    const bool act = k < P;
    const int r0 = act ? (int)(((unsigned)k * (unsigned)n) >> lgP) : 0;
    const int r1 = act ? (int)(((unsigned)(k + 1) * (unsigned)n) >> lgP) : 0;
    const int len = r1 - r0;
    // the line's component c (own order) in the grid's order
    auto gcomp = [](int c) -> int {
        if constexpr (NB == 4) return c == 1 ? NRM : (c == 2 ? 3 - NRM : c);
        else return c;
    };
    auto cell = [&](int c, int m) -> double {
        const int o = rev ? (n - 1 - m) : m;
        return sU[gcomp(c) * LP + padn<PSH>(o + kNG)];
    };
    auto rec = [&](int j, int q) -> double& { return scr[((long long)j * REC + q) * 64 + k]; };
    // closure values just outside a non-periodic line (explicit WENO5-Z per
    // component, as the component-wise path)
    double xlo[NB], xhi[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) xlo[c] = xhi[c] = 0.0;
    if (act && !cyclic && r0 == 0) {
#pragma unroll
        for (int c = 0; c < NB; ++c)
            xlo[c] = weno5z_value(cell(c, -3), cell(c, -2), cell(c, -1), cell(c, 0), cell(c, 1), weps);
    }
    if (act && !cyclic && r1 == n) {
#pragma unroll
        for (int c = 0; c < NB; ++c)
            xhi[c] = weno5z_value(cell(c, n - 2), cell(c, n - 1), cell(c, n), cell(c, n + 1),
                                  cell(c, n + 2), weps);
    }
    // Row gg of the block system in factored form: A = diag(ra) L,
    // B = diag(rb) L, C = diag(rc) L with L the left eigenvectors of the
    // node and (ra, rb, rc, rr) the scalar rows of eq. (CWENO-FV) of each
    // field; the closure values of a non-periodic line move to the right
    // side (ra or rc then 0).
    auto rows = [&](int gg, double (&L)[BB], double (&ra)[NB], double (&rb)[NB], double (&rc)[NB],
                    double (&r)[NB]) __attribute__((always_inline)) {
        double Ua[NB], Ub[NB], u5[5][NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            Ua[c] = cell(c, gg);
            Ub[c] = cell(c, gg + 1);
        }
        if constexpr (NB == 3) roe_left(gam, Ua, Ub, L);
        else roe_left4(gam, Ua, Ub, L);
#pragma unroll
        for (int m = 0; m < 5; ++m)
#pragma unroll
            for (int c = 0; c < NB; ++c) u5[m][c] = cell(c, gg - 2 + m);
#pragma unroll
        for (int f = 0; f < NB; ++f) {
            double v[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) v[m] = dotN<NB>(&L[NB * f], 1, u5[m], 1);
            double w0, w1, w2;
            wenoz_weights<double>(v[0], v[1], v[2], v[3], v[4], weps, w0, w1, w2);
            cweno_row<double>(w0, w1, w2, v[1], v[2], v[3], ra[f], rb[f], rc[f], r[f]);
        }
        if (!cyclic) {   // the known closure values move to the right side
            if (gg == 0) {
                double t[NB];
                mvN<NB>(L, xlo, t);
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    r[i] -= ra[i] * t[i];
                    ra[i] = 0.0;
                }
            }
            if (gg == n - 1) {
                double t[NB];
                mvN<NB>(L, xhi, t);
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    r[i] -= rc[i] * t[i];
                    rc[i] = 0.0;
                }
            }
        }
    };
    // forward chase: x_j = p_j + Q_j Lsep - Cp_j x_{j+1}.  The chunk's first
    // row in terms of the separators, x_{r0} = FP + FQ Lsep + FS Rsep, is
    // accumulated on the way: with M_0 = I and M_{j+1} = -M_j Cp_j,
    // FP = sum M_j p_j, FQ = sum M_j Q_j and FS = the last M; the rows'
    // (Cp, p, Q) go to the scratch for the recovery only.
    double cp[BB], pp[NB], qq[BB];
#pragma unroll
    for (int i = 0; i < BB; ++i) cp[i] = 0.0;
    set_identity<NB>(qq);
#pragma unroll
    for (int i = 0; i < NB; ++i) pp[i] = 0.0;
    double Ak[BB], Bk[BB], Ck[BB], Dk[NB];   // this lane's separator row
    double FP[NB], FQ[BB], FS[BB];   // first row: x_{r0} = FP + FQ Lsep + FS Rsep
#pragma unroll
    for (int i = 0; i < BB; ++i) {
        FQ[i] = 0.0;
        Ak[i] = 0.0;
        Ck[i] = 0.0;
    }
    set_identity<NB>(FS);
    set_identity<NB>(Bk);
#pragma unroll
    for (int i = 0; i < NB; ++i) Dk[i] = FP[i] = 0.0;
    double CX[BB];   // the separator row's coupling to the next chunk's first row
#pragma unroll
    for (int i = 0; i < BB; ++i) CX[i] = 0.0;
    if (act) {
        for (int j = 0; j < len - 1; ++j) {
            double L[BB], ra[NB], rb[NB], rc[NB], r[NB], M[BB], T[BB], Mi[BB], t3[NB];
            rows(r0 + j, L, ra, rb, rc, r);
            // M = B - A Cp = diag(rb) L - diag(ra) (L Cp)
            mmN<NB>(L, cp, T);
#pragma unroll
            for (int f = 0; f < NB; ++f)
#pragma unroll
                for (int q = 0; q < NB; ++q) M[NB * f + q] = rb[f] * L[NB * f + q] - ra[f] * T[NB * f + q];
            // r - A p
            mvN<NB>(L, pp, t3);
#pragma unroll
            for (int f = 0; f < NB; ++f) t3[f] = r[f] - ra[f] * t3[f];
            invN<NB>(M, Mi);
            // Cp = M^-1 C with C = diag(rc) L
#pragma unroll
            for (int f = 0; f < NB; ++f)
#pragma unroll
                for (int q = 0; q < NB; ++q) M[NB * f + q] = rc[f] * L[NB * f + q];
            mmN<NB>(Mi, M, cp);
            mvN<NB>(Mi, t3, pp);
            // Q = -M^-1 A Q_prev with A = diag(ra) L
            mmN<NB>(L, qq, T);
#pragma unroll
            for (int f = 0; f < NB; ++f)
#pragma unroll
                for (int q = 0; q < NB; ++q) T[NB * f + q] = -ra[f] * T[NB * f + q];
            mmN<NB>(Mi, T, qq);
#pragma unroll
            for (int i = 0; i < BB; ++i) {
                rec(j, i) = cp[i];
                rec(j, BB + NB + i) = qq[i];
            }
#pragma unroll
            for (int i = 0; i < NB; ++i) rec(j, BB + i) = pp[i];
            // FS holds M_j: FP += M_j p_j, FQ += M_j Q_j, then M_{j+1} = -M_j Cp_j
            mvN<NB>(FS, pp, t3);
#pragma unroll
            for (int i = 0; i < NB; ++i) FP[i] += t3[i];
            mmN<NB>(FS, qq, T);
#pragma unroll
            for (int i = 0; i < BB; ++i) FQ[i] += T[i];
            mmN<NB>(FS, cp, T);
#pragma unroll
            for (int i = 0; i < BB; ++i) FS[i] = -T[i];
        }
        // the chunk's last row, reduced onto the separators
        double L[BB], ra[NB], rb[NB], rc[NB], r[NB], T[BB], t3[NB];
        rows(r1 - 1, L, ra, rb, rc, r);
        mmN<NB>(L, qq, T);
#pragma unroll
        for (int f = 0; f < NB; ++f)
#pragma unroll
            for (int q = 0; q < NB; ++q) Ak[NB * f + q] = ra[f] * T[NB * f + q];
        mmN<NB>(L, cp, T);
#pragma unroll
        for (int f = 0; f < NB; ++f)
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                Bk[NB * f + q] = rb[f] * L[NB * f + q] - ra[f] * T[NB * f + q];
                CX[NB * f + q] = rc[f] * L[NB * f + q];
            }
        mvN<NB>(L, pp, t3);
#pragma unroll
        for (int f = 0; f < NB; ++f) Dk[f] = r[f] - ra[f] * t3[f];
    }
    // the next chunk's first-row relation (x_{r1} = FP' + FQ' Rsep + FS' Rsep')
    {
        const int kn = (k + 1) & (P - 1);
        double nP[NB], nQ[BB], nS[BB], T[BB], t3[NB];
        shflN<NB>(FP, kn, nP);
        shflN<BB>(FQ, kn, nQ);
        shflN<BB>(FS, kn, nS);
        mmN<NB>(CX, nQ, T);
#pragma unroll
        for (int i = 0; i < BB; ++i) Bk[i] += T[i];
        mmN<NB>(CX, nS, Ck);
        mvN<NB>(CX, nP, t3);
#pragma unroll
        for (int i = 0; i < NB; ++i) Dk[i] -= t3[i];
    }
    // block parallel cyclic reduction of the separator system over the wave;
    // the lower neighbour's blocks are used up before the upper one's are
    // fetched (the same arithmetic, fewer blocks live at once)
    for (int st = 1; st < P; st <<= 1) {
        const int km = (k - st) & (P - 1), kp = (k + st) & (P - 1);
        const bool lo_out = !cyclic && k - st < 0, hi_out = !cyclic && k + st >= P;
        double nA[BB], nB[BB], nD[NB], al[BB];
        {
            double Am[BB], Bm[BB], Cm[BB], Dm[NB], iBm[BB], T[BB], t3[NB];
            shflN<BB>(Ak, km, Am);
            shflN<BB>(Bk, km, Bm);
            shflN<BB>(Ck, km, Cm);
            shflN<NB>(Dk, km, Dm);
            if (lo_out) {
#pragma unroll
                for (int i = 0; i < BB; ++i) {
                    Am[i] = 0.0;
                    Cm[i] = 0.0;
                }
                set_identity<NB>(Bm);
#pragma unroll
                for (int i = 0; i < NB; ++i) Dm[i] = 0.0;
            }
            invN<NB>(Bm, iBm);
            mmN<NB>(Ak, iBm, al);
#pragma unroll
            for (int i = 0; i < BB; ++i) al[i] = -al[i];
            mmN<NB>(al, Cm, T);
#pragma unroll
            for (int i = 0; i < BB; ++i) nB[i] = Bk[i] + T[i];
            mvN<NB>(al, Dm, t3);
#pragma unroll
            for (int i = 0; i < NB; ++i) nD[i] = Dk[i] + t3[i];
            mmN<NB>(al, Am, nA);
        }
        {
            double Ap[BB], Bp[BB], Cp[BB], Dp[NB], iBp[BB], bt[BB], T[BB], t3[NB];
            shflN<BB>(Ak, kp, Ap);
            shflN<BB>(Bk, kp, Bp);
            shflN<BB>(Ck, kp, Cp);
            shflN<NB>(Dk, kp, Dp);
            if (hi_out) {
#pragma unroll
                for (int i = 0; i < BB; ++i) {
                    Ap[i] = 0.0;
                    Cp[i] = 0.0;
                }
                set_identity<NB>(Bp);
#pragma unroll
                for (int i = 0; i < NB; ++i) Dp[i] = 0.0;
            }
            invN<NB>(Bp, iBp);
            mmN<NB>(Ck, iBp, bt);
#pragma unroll
            for (int i = 0; i < BB; ++i) bt[i] = -bt[i];
            mmN<NB>(bt, Ap, T);
#pragma unroll
            for (int i = 0; i < BB; ++i) nB[i] += T[i];
            mvN<NB>(bt, Dp, t3);
#pragma unroll
            for (int i = 0; i < NB; ++i) nD[i] += t3[i];
            mmN<NB>(bt, Cp, Ck);
        }
#pragma unroll
        for (int i = 0; i < BB; ++i) {
            Ak[i] = nA[i];
            Bk[i] = nB[i];
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) Dk[i] = nD[i];
    }
    double Rs[NB], Ls[NB];
    {
        double M[BB], Mi[BB];
#pragma unroll
        for (int i = 0; i < BB; ++i) M[i] = cyclic ? Ak[i] + Bk[i] + Ck[i] : Bk[i];
        invN<NB>(M, Mi);
        mvN<NB>(Mi, Dk, Rs);
        shflN<NB>(Rs, (k - 1) & (P - 1), Ls);
        if (!cyclic && k == 0) {
#pragma unroll
            for (int i = 0; i < NB; ++i) Ls[i] = 0.0;
        }
    }
    if (act) {
        // recovery, last row first: x_j = p_j + Q_j Lsep - Cp_j x_{j+1}
        double xn[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            xn[i] = Rs[i];
            xs[(long long)gcomp(i) * n + r1 - 1] = Rs[i];
        }
        for (int j = len - 2; j >= 0; --j) {
            double cj[BB], pj[NB], qj[BB], x[NB], t3[NB];
#pragma unroll
            for (int i = 0; i < BB; ++i) {
                cj[i] = rec(j, i);
                qj[i] = rec(j, BB + NB + i);
            }
#pragma unroll
            for (int i = 0; i < NB; ++i) pj[i] = rec(j, BB + i);
            mvN<NB>(qj, Ls, t3);
#pragma unroll
            for (int i = 0; i < NB; ++i) x[i] = pj[i] + t3[i];
            mvN<NB>(cj, xn, t3);
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                x[i] -= t3[i];
                xs[(long long)gcomp(i) * n + r0 + j] = x[i];
                xn[i] = x[i];
            }
        }
    }
}

// Rows of the mixed system from the stored weights (w1 := 1 - w0 - w2 in
// float, so both passes see identical coefficients): eq. (CWENO-FV) matrix
// (a, b, c) and right-side weights (e0, e1, e2).
__device__ __forceinline__ void rows_from_w(float w0, float w2, float& a, float& b, float& c,
                                            float& e0, float& e1, float& e2) {
    const float w1 = 1.0f - w0 - w2;
    const float third = 1.0f / 3.0f, sixth = 1.0f / 6.0f;
    a = (2.0f * w0 + w1) * third;
    b = (w0 + 2.0f * (w1 + w2)) * third;
    c = w2 * third;
    e0 = w0 * sixth;
    e1 = (5.0f * (w0 + w1) + w2) * sixth;
    e2 = (w1 + 5.0f * w2) * sixth;
}

// One line (or one problem) through the whole operator.  NC components, NRM
// the normal momentum component, W waves per system (lines up to 2048 W),
// CPT cells per thread in phase 2, SEG1 = the line is one phase-2 segment,
// MIXED = float reconstruction/solve with one FP64-residual refinement
// sweep and a float HLLC (limiter and accumulation stay double).
// LOOPED: the caller runs line_op in a loop; the thread index is then passed
// through an empty asm so that values derived from it are recomputed per
// line rather than hoisted out of the loop and kept (spilled) across the solve.
// RECON: the reconstruction, PP_RECON_CWENO (the compact scheme) or one of the
// explicit comparison schemes (FP64 only; phase 1 then evaluates every face
// value from its own five averages and solves nothing).
// IFS (2D sweeps, FP64): reduce |u_n|+a over the averages and the limited
// interface states of the line into A.spd_if (the 2D interface-state rule).
template <int NC, int NRM, int W, int CPT, bool SEG1, bool MIXED, bool LOOPED = false,
          int RECON = PP_RECON_CWENO, bool IFS = false>
__device__ __forceinline__ void line_op(const LineArgs& A, int b, double* smem) {
    static_assert(RECON == PP_RECON_CWENO || !MIXED, "explicit schemes run in FP64");
    constexpr int NS = 2 * NC;
    constexpr int LANES = 64 * W;
    constexpr int NT = NS * LANES;
    // FP64 lines of up to 2048 cells: both sides of a component per lane
    constexpr bool PAIRED = !MIXED && W == 1 && RECON == PP_RECON_CWENO;
    constexpr int PSH = PAIRED ? 4 : 5;   // chunk stride 16 (paired) or 32 rows
    int tid = threadIdx.x;
    if constexpr (LOOPED) asm volatile("" : "+v"(tid));

    // ---- problem geometry
    const bool batched = A.off != nullptr;
    const int n = batched ? A.nline[b] : A.n;
    const double h = batched ? A.hline[b] : A.h;
    const int bc_lo = batched ? A.bcline[2 * b] : A.bc_lo;
    const int bc_hi = batched ? A.bcline[2 * b + 1] : A.bc_hi;
    const long long base = batched ? A.off[b] : (long long)b * A.ls;
    const bool cyclic = (bc_lo == PP_BC_PERIODIC);
    // stage epilogues (modes 1 and 2) and the time-step rules serve 1D lines
    // only: the 2D sweeps (NC = 4) write L (mode 0), and their kernels carry
    // none of that code
    constexpr bool kEpi = (NC == 3);
    // mode 4 (2D, FP64 compact scheme): write the face values before the
    // limiter for the Gauss-node operator, nothing else
    constexpr bool kFaces = (NC == 4) && !MIXED && RECON == PP_RECON_CWENO;
    const int mode = kEpi ? A.mode : ((kFaces && A.mode == 4) ? 4 : 0);
    // 2D interface-state rule: a separate instantiation of the compact
    // scheme's kernels (IFS), a run-time switch (A.spd_if) in the kernels of
    // the explicit and characteristic reconstructions
    constexpr bool kIfsRt = (NC == 4) && RECON != PP_RECON_CWENO;
    const bool ifs = IFS || (kIfsRt && A.spd_if != nullptr);
    const bool pprule = (kEpi && A.dtrule == PP_DT_PP) || (NC == 4 && ifs);
    double dt = 0.0;
    if (mode == 1) dt = batched ? A.dtline[b] : (A.dt_dev ? *A.dt_dev : A.dt_val);
    // mode 2 (stage 1 under the interface-state rule): dtline holds the time
    // left to t_end until this stage has chosen the step
    if (mode == 2 && batched) dt = A.dtline[b];
    if (batched && !(dt > 0.0)) return;  // finished problem: leave it untouched
    // status bits of a stage output go to the problem's word under the
    // restart rule (batched), else to the run's word
    unsigned* const stat = (batched && A.badline) ? &A.badline[b] : A.status;

    const double* __restrict__ U = A.U + base;
    const int LP = padn<PSH>(n + 2 * kNG - 1) + 1;   // padded LDS length of one component
    double* sU = smem;                          // phase 0/1: [NC][LP]
    // layout (same formula as the host): line data, then (W > 1 or paired) the
    // exchange scratch, and the reduction scratch after the largest area
    const long long area0 = (long long)NC * LP;
    const long long area1 = (W > 1 || !MIXED) ? (long long)NS * 512 : 0;
    const long long area2 = (long long)NS * (padn<PSH>(A.seg_max + 1) + 1);
    long long area = area0 + area1;
    area = area > area2 ? area : area2;
    double* sx = smem + area0;
    double* red = smem + area;

    // ---- phase 0: stage the line with ghosts; limiter epsilon
    double mr = INFINITY, me = INFINITY;
    for (int q = tid; q < n + 2 * kNG; q += NT) {
        const int i = q - kNG;   // cell index, -3..n+2
        int src;
        double sgn[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) sgn[c] = 1.0;
        if (i >= 0 && i < n) {
            src = i;
        } else if (cyclic) {
            src = (i + n) % n;
        } else {
            const int bc = i < 0 ? bc_lo : bc_hi;
            if (bc == PP_BC_TRANSMISSIVE) {
                src = i < 0 ? 0 : n - 1;
            } else {   // reflective: mirror image, normal momentum negated
                src = i < 0 ? (-i - 1) : (2 * n - 1 - i);
                src = src < 0 ? 0 : (src >= n ? n - 1 : src);
                sgn[NRM] = -1.0;
            }
        }
        double cell[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            cell[c] = U[(long long)c * A.cs + src];
            sU[c * LP + padn<PSH>(q)] = sgn[c] * cell[c];
        }
        if (i >= 0 && i < n && A.eps_enc == nullptr) {
            mr = fmin(mr, cell[0]);
            me = fmin(me, spec_e<NC>(cell));
        }
    }
    double eps_rho, eps_e;
    if (A.eps_enc != nullptr) {
        eps_rho = fmin(A.eps_cap, ord_dec(A.eps_enc[0]));
        eps_e = fmin(A.eps_cap, ord_dec(A.eps_enc[1]));
        __syncthreads();
    } else {
        block_min2<NT>(mr, me, red);   // contains the barriers
        eps_rho = fmin(A.eps_cap, mr);
        eps_e = fmin(A.eps_cap, me);
    }

    // ---- phase 1: chunked chasing of every (component, side) system.
    // PAIRED (FP64, lines <= 2048): one lane holds a chunk of BOTH systems of
    // its component, 128 lanes per component, so the smoothness indicators and
    // weight products of a cell are formed once for the two sides (the "+"
    // side at node j-1/2 of cell j uses the indicators of the "-" side at node
    // j+1/2 of the same cell, in mirrored order).  Otherwise one system per
    // 64 W lanes, the "+" system as the "-" system of the reversed line.
    constexpr int PL = PAIRED ? 128 : LANES;    // lanes per chunked system
    constexpr int CHP = kCHP;                   // paired: rows per lane and side
    const int sys = PAIRED ? 2 * (tid / 128) : tid / LANES;
    const int k = tid % PL;
    const int comp = sys >> 1;
    const bool rev = !PAIRED && (sys & 1) != 0;
    int P = PL, lgP = __builtin_ctz(PL);
    while (P > n) { P >>= 1; --lgP; }       // chunks: power of two, <= n
    const bool act = k < P;
    // chunk bounds floor(k n / P): lines hold at most 4096 cells and k <= P <=
    // 128, so the product fits 32 bits and the division is a shift
    const int r0 = act ? (int)(((unsigned)k * (unsigned)n) >> lgP) : 0;
    const int r1 = act ? (int)(((unsigned)(k + 1) * (unsigned)n) >> lgP) : 0;
    const int len = r1 - r0;
    const int knext = (k + 1) & (P - 1), kprev = (k - 1) & (P - 1);
    const double* sUc = sU + comp * LP;
    auto ub = [&](int m) -> double {
        const int o = rev ? (n - 1 - m) : m;
        return sUc[padn<PSH>(o + kNG)];
    };
    // closure of a non-periodic line (explicit WENO5-Z on the ghosts)
    double clo = 0.0, chi = 0.0;
    if (!PAIRED && act && !cyclic && r0 == 0)
        clo = weno5z_value(ub(-3), ub(-2), ub(-1), ub(0), ub(1), A.weno_eps);
    if (!PAIRED && act && !cyclic && r1 == n)
        chi = weno5z_value(ub(n - 2), ub(n - 1), ub(n), ub(n + 1), ub(n + 2), A.weno_eps);

    // per-lane results: x_j (double) = res(j)
    constexpr int CHE = PAIRED ? CHP : kCH;
    double E0[MIXED ? 1 : CHE], E1[MIXED ? 1 : CHE], E2[MIXED ? 1 : CHE];
    double F0[PAIRED ? CHP : 1], F1[PAIRED ? CHP : 1], F2[PAIRED ? CHP : 1];
    float X0[MIXED ? kCH : 1], Qf[MIXED ? kCH : 1], Sf[MIXED ? kCH : 1];
    float W0[MIXED ? kCH : 1], W2[MIXED ? kCH : 1];
    float Ld = 0.0f, Rd = 0.0f;   // mixed: separators of the correction solve

    if constexpr (PAIRED) {
        double* sxc = sx + comp * 1024;   // [8][128] exchange slots of this component
        if (n == kCHP * P)
            paired_solve<true>(sUc, n, k, P, cyclic, A.weno_eps, sxc, red + 4 * comp, r0, len, E0,
                               E1, E2, F0, F1, F2);
        else
            paired_solve<false>(sUc, n, k, P, cyclic, A.weno_eps, sxc, red + 4 * comp, r0, len, E0,
                                E1, E2, F0, F1, F2);
    } else if constexpr (RECON == PP_RECON_CHAR) {
        // characteristic-wise (FP64): waves 0 and 1 solve the block systems
        // of the "-" side and of the "+" side (the reversed line); every
        // (component, side) lane then takes its chunk of nodal values
        static_assert(!MIXED, "characteristic reconstruction runs in FP64");
        // this line's scratch: per line of a sweep, or per workgroup of a
        // persistent launch (each works one problem at a time)
        double* const chl = A.chs + (LOOPED ? (long long)blockIdx.x : (long long)b) * A.chs_line;
        double* const xsb = chl + 2 * A.chs_side;                  // [side][NC][n]
        if (tid < 128) {
            const int side = tid >> 6;
            char_side<NC, NRM, PSH>(sU, LP, n, cyclic, side == 1, tid & 63, A.gamma, A.weno_eps,
                                    chl + side * A.chs_side, xsb + (long long)side * NC * n);
        }
        __syncthreads();
        if (act) {
            const double* xsrc = xsb + (long long)(rev ? 1 : 0) * NC * n + (long long)comp * n;
#pragma unroll
            for (int j = 0; j < kCH; ++j)
                if (j < len) E0[j] = xsrc[r0 + j];
        }
    } else if constexpr (RECON != PP_RECON_CWENO) {
        // explicit scheme: x_g is the "-" value at node g+1/2 of this
        // system's (possibly reversed) line, from cells g-2 .. g+2
        if (act) {
#pragma unroll
            for (int j = 0; j < kCH; ++j) {
                if (j < len) {
                    const int g = r0 + j;
                    E0[j] = weno5_explicit<RECON == PP_RECON_WENOJS>(
                        ub(g - 2), ub(g - 1), ub(g), ub(g + 1), ub(g + 2), A.weno_eps);
                }
            }
        }
    } else if constexpr (!MIXED) {
        const double weps = A.weno_eps;
        double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;   // sliding window ubar_{g-2..g+1}
        if (act) {
            v0 = ub(r0 - 2);
            v1 = ub(r0 - 1);
            v2 = ub(r0);
            v3 = ub(r0 + 1);
        }
        auto row = [&](int j, double& a, double& bb, double& c, double& r) {
            const int g = r0 + j;
            const double v4 = ub(g + 2);
            double w0, w1, w2;
            wenoz_weights<double>(v0, v1, v2, v3, v4, weps, w0, w1, w2);
            cweno_row<double>(w0, w1, w2, v1, v2, v3, a, bb, c, r);
            if (!cyclic) {
                if (g == 0) { r -= a * clo; a = 0.0; }
                if (g == n - 1) { r -= c * chi; c = 0.0; }
            }
            v0 = v1; v1 = v2; v2 = v3; v3 = v4;
        };
        chunk_chase_solve<W>(row, act, k, P, len, cyclic, sx, sys, E0, E1, E2);
    } else {
        // ---------------- pass A: float weights, rows and chasing
        float ae = 0.0f, be = 1.0f, ce = 0.0f, re = 0.0f;
        float gP = 0.0f, gQ = 1.0f, gS = 0.0f, fP = 0.0f, fQ = 0.0f, fS = 1.0f;
        const float weps = (float)A.weno_eps;
        if (act) {
            float v0 = (float)ub(r0 - 2), v1 = (float)ub(r0 - 1), v2 = (float)ub(r0),
                  v3 = (float)ub(r0 + 1);
            float cprev = 0.0f, pprev = 0.0f, qprev = 0.0f;
#pragma unroll
            for (int j = 0; j < kCH; ++j) {
                if (j < len) {
                    const int g = r0 + j;
                    const float v4 = (float)ub(g + 2);
                    float w0, w1, w2, a, bb, c, e0, e1, e2;
                    wenoz_weights<float>(v0, v1, v2, v3, v4, weps, w0, w1, w2);
                    W0[j] = w0;
                    W2[j] = w2;
                    rows_from_w(w0, w2, a, bb, c, e0, e1, e2);
                    float r = e0 * v1 + e1 * v2 + e2 * v3;
                    if (!cyclic) {
                        if (g == 0) { r -= a * (float)clo; a = 0.0f; }
                        if (g == n - 1) { r -= c * (float)chi; c = 0.0f; }
                    }
                    if (j < len - 1) {
                        const float piv = (j == 0) ? bb : bb - a * cprev;
                        const float ip = rcp_t(piv);
                        const float cj = c * ip;
                        const float pj = ((j == 0) ? r : r - a * pprev) * ip;
                        const float qj = ((j == 0) ? -a : -a * qprev) * ip;
                        X0[j] = cj; Qf[j] = pj; Sf[j] = qj;
                        cprev = cj; pprev = pj; qprev = qj;
                    } else {
                        ae = a; be = bb; ce = c; re = r;
                    }
                    v0 = v1; v1 = v2; v2 = v3; v3 = v4;
                }
            }
            float Pn = 0.0f, Qn = 0.0f, Sn = 0.0f;
#pragma unroll
            for (int j = kCH - 1; j >= 0; --j) {
                if (j < len - 1) {
                    const float cj = X0[j];
                    float Pj, Qj, Sj;
                    if (j == len - 2) {
                        Pj = Qf[j]; Qj = Sf[j]; Sj = -cj;
                        gP = Pj; gQ = Qj; gS = Sj;
                    } else {
                        Pj = Qf[j] - cj * Pn; Qj = Sf[j] - cj * Qn; Sj = -cj * Sn;
                    }
                    X0[j] = Pj; Qf[j] = Qj; Sf[j] = Sj;
                    Pn = Pj; Qn = Qj; Sn = Sj;
                }
            }
            if (len >= 2) { fP = X0[0]; fQ = Qf[0]; fS = Sf[0]; }
        }
        double nf[3] = {fP, fQ, fS};
        xch<W, 3>(nf, knext, sx, sys, k);
        if (!cyclic && k + 1 >= P) nf[0] = nf[1] = nf[2] = 0.0;
        const float RA = ae * gQ, RB = be + ae * gS + ce * (float)nf[1], RC = ce * (float)nf[2];
        const float R0 = pcr_solve<W, float>(RA, RB, RC, re - ae * gP - ce * (float)nf[0], k, P,
                                             cyclic, sx, sys);
        double lv[1] = {(double)R0};
        xch<W, 1>(lv, kprev, sx, sys, k);
        const float L0 = (!cyclic && k == 0) ? 0.0f : (float)lv[0];
        if (act) {
#pragma unroll
            for (int j = 0; j < kCH; ++j) {
                if (j < len - 1) X0[j] = X0[j] + Qf[j] * L0 + Sf[j] * R0;
                else if (j == len - 1) X0[j] = R0;
            }
        }
        // ---------------- refinement sweep: FP64 residual of the float
        // system, float correction through the same chunk factorisation
        double xn[1] = {act && len >= 1 ? (double)X0[0] : 0.0};   // next chunk's x_{r0}
        xch<W, 1>(xn, knext, sx, sys, k);
        float ge = 0.0f, fe = 0.0f;     // P parts of x_{r1-2} and x_{r0}
        float res_e = 0.0f;             // residual of the separator row
        if (act) {
            double v1 = ub(r0 - 1), v2 = ub(r0), v3 = ub(r0 + 1);
            float cprev = 0.0f, pprev = 0.0f;
            double xm = (double)L0;     // x_{g-1}
#pragma unroll
            for (int j = 0; j < kCH; ++j) {
                if (j < len) {
                    const int g = r0 + j;
                    // float rows: the factorisation of pass A; double rows
                    // (same float weights): the system whose residual is taken
                    float a, bb, c, e0, e1, e2;
                    rows_from_w(W0[j], W2[j], a, bb, c, e0, e1, e2);
                    const double dw0 = (double)W0[j], dw2 = (double)W2[j];
                    const double dw1 = 1.0 - dw0 - dw2;
                    // the row times 6 (exact scalings only), residual scaled back
                    double da = 2.0 * (2.0 * dw0 + dw1), db = 2.0 * (dw0 + 2.0 * (dw1 + dw2));
                    double dc = 2.0 * dw2;
                    double r = dw0 * v1 + (5.0 * (dw0 + dw1) + dw2) * v2 + (dw1 + 5.0 * dw2) * v3;
                    if (!cyclic) {
                        if (g == 0) { r -= da * clo; da = 0.0; a = 0.0f; }
                        if (g == n - 1) { r -= dc * chi; dc = 0.0; c = 0.0f; }
                    }
                    const double x0 = (double)X0[j];
                    const double xp = (j + 1 < len) ? (double)X0[j + 1 < kCH ? j + 1 : kCH - 1]
                                                    : xn[0];
                    const double res = (r - (da * xm + db * x0 + dc * xp)) * (1.0 / 6.0);
                    const float rf = (float)res;
                    if (j < len - 1) {
                        const float piv = (j == 0) ? bb : bb - a * cprev;
                        const float ip = rcp_t(piv);
                        const float cj = c * ip;
                        const float pj = ((j == 0) ? rf : rf - a * pprev) * ip;
                        W0[j] = cj;
                        W2[j] = pj;
                        cprev = cj;
                        pprev = pj;
                    } else {
                        res_e = rf;
                    }
                    xm = x0;
                    v1 = v2;
                    v2 = v3;
                    v3 = ub(g + 2);
                }
            }
            float Pn = 0.0f;
#pragma unroll
            for (int j = kCH - 1; j >= 0; --j) {
                if (j < len - 1) {
                    const float Pj = (j == len - 2) ? W2[j] : W2[j] - W0[j] * Pn;
                    W2[j] = Pj;
                    Pn = Pj;
                    if (j == len - 2) ge = Pj;
                }
            }
            if (len >= 2) fe = W2[0];
        }
        double nfe[1] = {(double)fe};
        xch<W, 1>(nfe, knext, sx, sys, k);
        if (!cyclic && k + 1 >= P) nfe[0] = 0.0;
        Rd = pcr_solve<W, float>(RA, RB, RC, res_e - ae * ge - ce * (float)nfe[0], k, P, cyclic,
                                 sx, sys);
        double ld[1] = {(double)Rd};
        xch<W, 1>(ld, kprev, sx, sys, k);
        Ld = (!cyclic && k == 0) ? 0.0f : (float)ld[0];
    }
    __syncthreads();   // line data and exchange scratch done: LDS becomes staging

    // ---- phase 2: limiter, HLLC, flux difference, epilogue (by segments)
    const int SMAX = A.seg_max;
    const int SS = padn<PSH>(SMAX + 1) + 1;
    double* sRes = smem;                         // [NS][SS], slots padded
    double smax_speed = 0.0;
    double smax_if = 0.0;   // interface-state rule: |u|+a over averages and limited states
    unsigned bad = 0u;
    // SEG1: the whole line is one segment (the loop disappears at compile time)
    const int nseg = SEG1 ? 1 : (n + SMAX - 1) / SMAX;
    for (int sg = 0; sg < nseg; ++sg) {
        const int g0 = sg * SMAX;
        const int g1 = min(n, g0 + SMAX);
        const int S = g1 - g0;
        const int left = cyclic ? (g0 - 1 + n) % n : g0 - 1;
        const int right = cyclic ? g1 % n : g1;
        static_assert(kCHP == 16, "the paired path pads one slot per 16 rows");
        if (PAIRED && SEG1 && act && n == kCHP * P) {
            // every lane holds 16 cells of the one segment: slot padn<4>(16 k
            // + j + 1) = 17 k + padn<4>(j + 1); periodic ghost slots 0 and
            // n + 1 take cells n - 1 (last lane) and 0 (lane 0)
            double* rowm = sRes + (2 * comp) * SS;
            double* rowp = rowm + SS;
            double* bm = rowm + 17 * k;
            double* bp = rowp + 17 * k;
#pragma unroll
            for (int j = 0; j < CHP; ++j) {
                bm[padn<4>(j + 1)] = E0[j];
                bp[padn<4>(j + 1)] = F0[j];
            }
            if (cyclic && k == 0) {
                rowm[padn<4>(n + 1)] = E0[0];
                rowp[padn<4>(n + 1)] = F0[0];
            }
            if (cyclic && k == P - 1) {
                rowm[0] = E0[CHP - 1];
                rowp[0] = F0[CHP - 1];
            }
            if (A.dbg_um) {
#pragma unroll
                for (int j = 0; j < CHP; ++j) A.dbg_um[(long long)comp * n + r0 + j] = E0[j];
            }
            if (A.dbg_up) {
#pragma unroll
                for (int j = 0; j < CHP; ++j) A.dbg_up[(long long)comp * n + r0 + j] = F0[j];
            }
        } else if (PAIRED && act) {
            double* rowm = sRes + (2 * comp) * SS;
            double* rowp = rowm + SS;
#pragma unroll
            for (int j = 0; j < CHP; ++j) {
                if (j < len) {
                    const int cell = r0 + j;
                    const double xm = E0[j], xp = F0[j];
                    if (cell >= g0 && cell < g1) {
                        rowm[padn<PSH>(cell - g0 + 1)] = xm;
                        rowp[padn<PSH>(cell - g0 + 1)] = xp;
                        if (A.dbg_um) A.dbg_um[(long long)comp * n + cell] = xm;
                        if (A.dbg_up) A.dbg_up[(long long)comp * n + cell] = xp;
                    }
                    if (cell == left) { rowm[0] = xm; rowp[0] = xp; }
                    if (cell == right) {
                        rowm[padn<PSH>(S + 1)] = xm;
                        rowp[padn<PSH>(S + 1)] = xp;
                    }
                }
            }
        } else if (act) {
#pragma unroll
            for (int j = 0; j < kCH; ++j) {
                if (j < len) {
                    const int g = r0 + j;
                    const int cell = rev ? (n - 1 - g) : g;
                    // x_j of this lane's chunk, in double
                    double x;
                    if constexpr (MIXED) {
                        const float d = (j < len - 1) ? W2[j] + Qf[j] * Ld + Sf[j] * Rd : Rd;
                        x = (double)X0[j] + (double)d;
                    } else {
                        x = E0[j];
                    }
                    double* row = sRes + sys * SS;
                    if (cell >= g0 && cell < g1) {
                        row[padn<PSH>(cell - g0 + 1)] = x;
                        double* d = rev ? A.dbg_up : A.dbg_um;
                        if (d) d[(long long)comp * n + cell] = x;
                    }
                    if (cell == left) row[0] = x;
                    if (cell == right) row[padn<PSH>(S + 1)] = x;
                }
            }
        }
        __syncthreads();
        if (kFaces && mode == 4) {
            // face values of cells g0 .. g1-1: planes c (U- at the right face)
            // and NC + c (U+ at the left face) of out
            for (int q = tid; q < NC * S; q += NT) {
                const int c = q / S, r = q - c * S;
                const long long at = base + (long long)c * A.cs + g0 + r;
                A.out[at] = sRes[(2 * c) * SS + padn<PSH>(r + 1)];
                A.out[at + (long long)NC * A.cs] = sRes[(2 * c + 1) * SS + padn<PSH>(r + 1)];
            }
            __syncthreads();
            continue;
        }
        // limiter on slots 0..S+1 (cells g0-1 .. g1); a single segment reads its
        // edge neighbours from slots S and 1 instead (periodic) or not at all
        for (int q = tid + (SEG1 ? 1 : 0); q < S + (SEG1 ? 1 : 2); q += NT) {
            const int cell = (q == 0) ? left : (q == S + 1 ? right : g0 + q - 1);
            if (cell < 0 || cell >= n) continue;
            double Ub[NC], Um[NC], Up[NC];
            const int pq = padn<PSH>(q);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                Ub[c] = U[(long long)c * A.cs + cell];
                Um[c] = sRes[(2 * c) * SS + pq];
                Up[c] = sRes[(2 * c + 1) * SS + pq];
            }
            pp_limit<NC, NRM>(A.w1, A.i12, eps_rho, eps_e, Ub, Um, Up);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                sRes[(2 * c) * SS + pq] = Um[c];
                sRes[(2 * c + 1) * SS + pq] = Up[c];
            }
            if (pprule) {
                // sup-norm of |u|+a over the averages and the limited
                // interface states (condition (CFL-CD)); a non-finite speed
                // makes the bound infinite, so no step is taken
                const double sp = fmax(wave_speed<NC, NRM>(A.gamma, Ub),
                                       fmax(wave_speed<NC, NRM>(A.gamma, Um),
                                            wave_speed<NC, NRM>(A.gamma, Up)));
                smax_if = isfinite(sp) ? fmax(smax_if, sp) : INFINITY;
            }
        }
        __syncthreads();
        // fluxes: face f = g0 + r (between cells f-1 and f), r = 0..S, strided
        // over the threads; a single segment of a periodic line skips face 0,
        // which is face n
        auto face = [&](int f, double (&F)[NC]) {
            double Ul[NC], Ur[NC];
            int ql = f - g0, qr = f - g0 + 1;   // slots of cells f-1 and f
            if (SEG1 && cyclic) {
                if (f == 0) ql = S;
                if (f == n) qr = 1;
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                Ul[c] = sRes[(2 * c) * SS + padn<PSH>(ql)];
                Ur[c] = sRes[(2 * c + 1) * SS + padn<PSH>(qr)];
            }
            if (!cyclic && f == 0) {
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    Ul[c] = (bc_lo == PP_BC_REFLECTIVE && c == NRM) ? -Ur[c] : Ur[c];
            }
            if (!cyclic && f == n) {
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    Ur[c] = (bc_hi == PP_BC_REFLECTIVE && c == NRM) ? -Ul[c] : Ul[c];
            }
            if (A.flux == PP_FLUX_LF) {
                lf_flux<NC, NRM>(A.gamma, Ul, Ur, F);   // double in both precisions
            } else if constexpr (MIXED) {
                hllc_flux_f32<NC, NRM>(A.gamma, Ul, Ur, F);
            } else {
                hllc_flux<NC, NRM>(A.gamma, Ul, Ur, F);
            }
            if (A.dbg_flux) {
#pragma unroll
                for (int c = 0; c < NC; ++c) A.dbg_flux[(long long)c * (n + 1) + f] = F[c];
            }
        };
        const bool wrap0 = SEG1 && cyclic;
        const int r_lo = wrap0 ? 1 : 0;
        constexpr int KF = CPT + 1;   // faces per thread at most
        double Fr[KF][NC];
#pragma unroll
        for (int kk = 0; kk < KF; ++kk) {
            const int r = r_lo + tid + kk * NT;
            if (r <= S) face(g0 + r, Fr[kk]);
        }
        __syncthreads();   // staging reads done: the flux table takes its place
        double* sF = smem;   // [NC][S + 1]
        const int FS = S + 1;
#pragma unroll
        for (int kk = 0; kk < KF; ++kk) {
            const int r = r_lo + tid + kk * NT;
            if (r <= S) {
#pragma unroll
                for (int c = 0; c < NC; ++c) sF[c * FS + r] = Fr[kk][c];
            }
        }
        __syncthreads();
        // flux difference and epilogue, cells strided over the threads so the
        // global loads and stores are coalesced
        const double ih = 1.0 / h;
        for (int q = tid; q < S; q += NT) {
            const int i = g0 + q;
            double o[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double Fl = sF[c * FS + ((wrap0 && q == 0) ? S : q)];
                const double L = -(sF[c * FS + q + 1] - Fl) * ih;
                if (wrap0 && q == 0 && A.dbg_flux) A.dbg_flux[(long long)c * (n + 1)] = Fl;
                const long long at = base + (long long)c * A.cs + i;
                if (mode != 1) {
                    o[c] = L;
                } else {
                    const double us = A.U[at];
                    const double u0 = (A.rk_a != 0.0) ? A.U0[at] : 0.0;
                    o[c] = A.rk_a * u0 + A.rk_b * (us + dt * L);
                }
                // 2D x-sweep: L_x goes out past the caches (the y-sweep
                // streams the whole state before the combine reads it);
                // L_y stays cacheable for the combine that follows at once
                if constexpr (NC == 4 && NRM == 1) __builtin_nontemporal_store(o[c], &A.out[at]);
                else A.out[at] = o[c];
            }
            if (mode == 1) {
                // state checks without divisions: rho > 0 and rho E - |m|^2/2 > 0
                double m2 = 0.0;
#pragma unroll
                for (int c = 1; c < NC - 1; ++c) m2 += o[c] * o[c];
                bool fin = true;
#pragma unroll
                for (int c = 0; c < NC; ++c) fin = fin && isfinite(o[c]);
                if (!fin) bad |= 1u;
                if (!(o[0] > 0.0) || !(o[0] * o[NC - 1] - 0.5 * m2 > 0.0)) bad |= 2u;
                if (A.stage == 3) smax_speed = fmax(smax_speed, wave_speed<NC, NRM>(A.gamma, o));
            }
        }
        __syncthreads();
    }
    if constexpr (NC == 4 && (IFS || kIfsRt)) {
        if (ifs) {   // uniform over the block
            const double S = block_max<NT>(smax_if, red);
            if (tid == 0) atomicMax(A.spd_if, ord_enc(S));
        }
    }
    if (mode == 2) {
        // stage 1 under the interface-state rule: the step's dt from the
        // sup-norm over this stage input, then U1 = U + dt L over the L just
        // written (same rounding as the one-pass stage 1)
        const double S = block_max<NT>(smax_if, red);
        if (tid == 0) {
            double d = A.cfl * h / S;
            const double rem = batched ? dt : (A.scal ? A.t_end - A.scal->t : 0.0);
            if (!(d > 0.0) || !isfinite(d)) {
                d = 0.0;
                if (A.status) atomicOr(A.status, 1u);
            } else if (d > rem) {
                d = rem;
            }
            if (batched) {
                A.dtline[b] = d;
            } else if (A.scal) {
                A.scal->dt = d;
                if (!(d > 0.0)) A.scal->active = 0;
            }
            red[0] = d;
        }
        __syncthreads();
        const double d = red[0];
        __syncthreads();
        if (d > 0.0) {
            for (int q = tid; q < n; q += NT) {
                double o[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const long long at = base + (long long)c * A.cs + q;
                    o[c] = A.U[at] + d * A.out[at];
                    A.out[at] = o[c];
                }
                double m2 = 0.0;
#pragma unroll
                for (int c = 1; c < NC - 1; ++c) m2 += o[c] * o[c];
                bool fin = true;
#pragma unroll
                for (int c = 0; c < NC; ++c) fin = fin && isfinite(o[c]);
                if (!fin) bad |= 1u;
                if (!(o[0] > 0.0) || !(o[0] * o[NC - 1] - 0.5 * m2 > 0.0)) bad |= 2u;
            }
            if (bad && stat) atomicOr(stat, bad);
        }
    }
    if (mode == 1) {
        if (pprule && A.stage >= 2) {
            // the stage input against condition (CFL-CD) with the step's dt
            const double S = block_max<NT>(smax_if, red);
            if (dt * S > A.w1 * h) bad |= 4u;
        }
        if (bad && stat) atomicOr(stat, bad);
        if (A.stage == 3) {
            const double S = block_max<NT>(smax_speed, red);
            if (batched) {
                unsigned sbad = 0u;
                if (A.badline) {
                    // restart rule: the step of this problem stands only if no
                    // stage output left G; then the stage-3 output (in out) is
                    // copied into the state, else the step is redone with half
                    // the dt.  The word collects the bits of all three stages.
                    if (tid == 0)
                        red[0] = (double)__hip_atomic_load(&A.badline[b], __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                    __syncthreads();
                    sbad = (unsigned)red[0];
                    __syncthreads();
                    if (sbad == 0u) {
                        for (int q = tid; q < n; q += NT) {
#pragma unroll
                            for (int c = 0; c < NC; ++c) {
                                const long long at = base + (long long)c * A.cs + q;
                                A.commit[at] = A.out[at];
                            }
                        }
                    }
                }
                if (tid == 0) {
                    double dn;
                    if (sbad != 0u) {
                        // redo this step from U^n with half the dt
                        const int hv = A.halfline[b] + 1;
                        A.halfline[b] = hv;
                        const double t = A.tline[b];
                        if (hv > kMaxHalvings || t + 0.5 * dt == t) {   // or a stall
                            dn = 0.0;
                            if (A.status) atomicOr(A.status, sbad);
                        } else {
                            dn = 0.5 * dt;
                            atomicAdd(A.restart_count, 1ull);
                        }
                        A.badline[b] = 0u;
                    } else {
                        // next step of this problem: dt = cfl h / max(|u|+a) of
                        // the new averages (interface-state rule: the time left,
                        // the next stage 1 picks dt), clipped to t_end; 0
                        // retires the problem
                        const double t = A.tline[b] + dt;
                        const long long st = A.stepline[b] + 1;
                        A.tline[b] = t;
                        A.stepline[b] = st;
                        if (A.badline) {
                            A.halfline[b] = 0;
                            A.badline[b] = 0u;
                        }
                        if (pprule) {
                            dn = A.t_end - t;
                        } else {
                            dn = A.cfl * h / S;
                            if (!(dn > 0.0) || !isfinite(dn)) {
                                dn = 0.0;
                                if (A.status) atomicOr(A.status, 1u);
                            }
                        }
                        if (t >= A.t_end || st >= A.steps_max) dn = 0.0;
                        else if (t + dn > A.t_end) dn = A.t_end - t;
                    }
                    A.dtline[b] = dn;
                }
            } else if (A.scal && tid == 0) {
                atomicMax(&A.scal->spd[0], ord_enc(S));
            }
        }
    }
}

template <int NC, int NRM, int W, int CPT, bool SEG1, bool MIXED, int RECON = PP_RECON_CWENO,
          bool IFS = false>
__global__ void __launch_bounds__(2 * NC * 64 * W) line_kernel(LineArgs A) {
    extern __shared__ double smem[];
    if (A.scal && !A.scal->active) return;
    line_op<NC, NRM, W, CPT, SEG1, MIXED, false, RECON, IFS>(A, blockIdx.x, smem);
}

// Batched ensemble: one persistent launch per stage; workgroups pop problem
// ids (longest first) from a counter until the queue is empty.
template <int NC, int NRM, int W, int CPT, bool SEG1, bool MIXED, int RECON = PP_RECON_CWENO>
__global__ void __launch_bounds__(2 * NC * 64 * W) line_kernel_persistent(LineArgs A) {
    extern __shared__ double smem[];
    __shared__ int next;
    typedef __attribute__((address_space(4))) const LineArgs KArgs;
    for (;;) {
        // the arguments are re-read from the kernel-argument segment for every
        // problem (the empty asm hides that they are loop invariant), so they
        // are not hoisted into registers that would live across the solve
        KArgs* ap = (KArgs*)__builtin_amdgcn_kernarg_segment_ptr();
        asm volatile("" : "+s"(ap));
        const LineArgs& Ai = *(const LineArgs*)ap;
        if (threadIdx.x == 0) next = atomicAdd(Ai.counter, 1);
        __syncthreads();
        const int q = next;
        __syncthreads();
        if (q >= Ai.nlines) break;
        line_op<NC, NRM, W, CPT, SEG1, MIXED, true, RECON>(Ai, Ai.order[q], smem);
        __syncthreads();
    }
}

__global__ void reset_counter(int* c) { *c = 0; }

// Batched run start: per problem t = 0, steps = 0 and the first dt from the
// wave speeds of its initial averages.
__global__ void __launch_bounds__(256) batch_init_kernel(const double* __restrict__ U,
                                                         long long total, const long long* off,
                                                         const int* nl, const double* hl,
                                                         double* dtl, double* tl, long long* sl,
                                                         double gamma, double cfl, double t_end,
                                                         int resume, long long steps_max,
                                                         int rule, unsigned* badl, int* halfl) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    const long long o = off[b];
    double S = 0.0;
    for (int i = threadIdx.x; i < nl[b]; i += 256) {
        const double q[3] = {U[o + i], U[total + o + i], U[2 * total + o + i]};
        S = fmax(S, wave_speed<3, 1>(gamma, q));
    }
#pragma unroll
    for (int k = 32; k > 0; k >>= 1) S = fmax(S, __shfl_xor(S, k));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = S;
    __syncthreads();
    if (threadIdx.x == 0) {
        S = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        // the interface-state rule keeps the time left to t_end here; its
        // stage 1 picks the step
        double dt = rule == PP_DT_PP ? t_end - (resume ? tl[b] : 0.0) : cfl * hl[b] / S;
        if (badl) {
            badl[b] = 0u;
            halfl[b] = 0;
        }
        if (!resume) {
            if (!(dt > 0.0) || !isfinite(dt)) dt = 0.0;
            if (dt > t_end) dt = t_end;
            tl[b] = 0.0;
            sl[b] = 0;
        } else {
            // continue from the stored t and step count with the dt the
            // stage-3 epilogue would have set (same averages, same rule)
            const double t = tl[b];
            if (!(dt > 0.0) || !isfinite(dt) || t >= t_end || sl[b] >= steps_max) dt = 0.0;
            else if (t + dt > t_end) dt = t_end - t;
        }
        dtl[b] = dt;
    }
}

// ---------------------------------------------------------------- 2D pieces
constexpr int TT = 32;   // transpose tile edge

// B[c][x][y] = A[c][y][x]
__global__ void __launch_bounds__(256) transpose_kernel(const double* __restrict__ src,
                                                        double* __restrict__ dst, int nx, int ny,
                                                        int ncomp) {
    __shared__ double tile[TT][TT + 1];
    const long long cs = (long long)nx * ny;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int x0 = blockIdx.x * TT, y0 = blockIdx.y * TT;
    for (int c = 0; c < ncomp; ++c) {
        for (int yy = ty; yy < TT; yy += 8) {
            const int x = x0 + tx, y = y0 + yy;
            if (x < nx && y < ny) tile[yy][tx] = src[c * cs + (long long)y * nx + x];
        }
        __syncthreads();
        for (int xx = ty; xx < TT; xx += 8) {
            const int y = y0 + tx, x = x0 + xx;
            if (x < nx && y < ny) dst[c * cs + (long long)x * ny + y] = tile[tx][xx];
        }
        __syncthreads();
    }
}

// mode 0: Out = Lx + Ly (L only).  mode 1: Out = a Un + b (Us + dt (Lx + Ly)),
// written in layout A (Out) and B (OutB); reduces min rho / min e of the
// output into eps_out and (stage 3) max speeds into spd_out.  64x64 tiles,
// one component at a time, 1024 threads; every array is read and written in
// 512-byte runs (a wave covers 64 consecutive doubles of one row).
constexpr int TC = 64;
__global__ void __launch_bounds__(1024) combine2d_kernel(
    const double* __restrict__ Lx, const double* __restrict__ LyB, const double* __restrict__ Us,
    const double* Un, double* Out, double* __restrict__ OutB, int nx,
    int ny, int mode, double ra, double rb, const double* dt_dev, double dt_val, double gamma,
    long long* eps_out, long long* spd_out, long long* eps_reset, Scal* scal, unsigned* status) {
    __shared__ double tile[TC][TC + 1];
    __shared__ double red[16][4];
    if (scal && !scal->active) return;
    if (eps_reset && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        eps_reset[0] = kEncPosInf;
        eps_reset[1] = kEncPosInf;
    }
    const long long cs = (long long)nx * ny;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int x0 = blockIdx.x * TC, y0 = blockIdx.y * TC;
    const double dt = dt_dev ? *dt_dev : dt_val;
    const bool rd0 = mode == 1 && ra != 0.0;
    double cell[4][4];   // [row][comp] of this thread's cells (x0 + tx, y0 + ty + 16 r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double lx[4], us[4], un[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int xx = ty + 16 * r;
            const int y = y0 + tx, x = x0 + xx;
            if (x < nx && y < ny)
                tile[xx][tx] = __builtin_nontemporal_load(&LyB[c * cs + (long long)x * ny + y]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int x = x0 + tx, y = y0 + ty + 16 * r;
            lx[r] = us[r] = un[r] = 0.0;
            if (x < nx && y < ny) {
                const long long at = c * cs + (long long)y * nx + x;
                lx[r] = __builtin_nontemporal_load(&Lx[at]);
                if (mode == 1) us[r] = __builtin_nontemporal_load(&Us[at]);
                if (rd0) un[r] = __builtin_nontemporal_load(&Un[at]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int yy = ty + 16 * r;
            const int x = x0 + tx, y = y0 + yy;
            const double L = lx[r] + tile[tx][yy];
            const double v = (mode == 0) ? L : ra * un[r] + rb * (us[r] + dt * L);
            if (x < nx && y < ny) __builtin_nontemporal_store(v, &Out[c * cs + (long long)y * nx + x]);
            cell[r][c] = v;
        }
        __syncthreads();   // tile reads done
        if (mode == 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) tile[ty + 16 * r][tx] = cell[r][c];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int xx = ty + 16 * r;
                const int y = y0 + tx, x = x0 + xx;
                if (x < nx && y < ny)
                    __builtin_nontemporal_store(tile[tx][xx], &OutB[c * cs + (long long)x * ny + y]);
            }
            __syncthreads();   // before the next component's tile
        }
    }
    if (mode != 1) return;
    double mr = INFINITY, me = INFINITY, sx = 0.0, sy = 0.0;
    unsigned bad = 0u;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int x = x0 + tx, y = y0 + ty + 16 * r;
        if (x >= nx || y >= ny) continue;
        const double q[4] = {cell[r][0], cell[r][1], cell[r][2], cell[r][3]};
        const double e = spec_e<4>(q);
        mr = fmin(mr, q[0]);
        me = fmin(me, e);
        const double p = (gamma - 1.0) * q[0] * e;
        if (!(isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && isfinite(q[3]))) bad |= 1u;
        if (!(q[0] > 0.0) || !(p > 0.0)) bad |= 2u;
        if (spd_out) {
            sx = fmax(sx, wave_speed<4, 1>(gamma, q));
            sy = fmax(sy, wave_speed<4, 2>(gamma, q));
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mr = fmin(mr, __shfl_xor(mr, o));
        me = fmin(me, __shfl_xor(me, o));
        sx = fmax(sx, __shfl_xor(sx, o));
        sy = fmax(sy, __shfl_xor(sy, o));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = mr; red[w][1] = me; red[w][2] = sx; red[w][3] = sy;
    }
    if (bad && status) atomicOr(status, bad);
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 16; ++i) {
            mr = fmin(mr, red[i][0]); me = fmin(me, red[i][1]);
            sx = fmax(sx, red[i][2]); sy = fmax(sy, red[i][3]);
        }
        atomicMin(&eps_out[0], ord_enc(mr));
        atomicMin(&eps_out[1], ord_enc(me));
        if (spd_out) {
            atomicMax(&spd_out[0], ord_enc(sx));
            atomicMax(&spd_out[1], ord_enc(sy));
        }
    }
}

// ----------------------------------------------------- Gauss-node 2D operator
// Face fluxes averaged over each face by three-point Gauss-Legendre quadrature
// (a multi-dimensional form the paper leaves to future work, Sec. 4).  The
// line kernel in mode 4 writes every cell's two face values before the
// limiter (averages over the cell's transverse extent, from the compact
// reconstruction of Sec. 2.2); this kernel turns the face values of five
// neighbouring lines into values at the face's Gauss nodes, limits a cell's
// six node states as the steps of Sec. 2.4 do, and sums the node fluxes.

// value at Gauss node k of a face = sum_m c[k][m] x (face value of line l-2+m);
// g[k] the Gauss-Legendre weights
struct GaussCoef {
    double c[3][5];
    double g[3];
};

constexpr int kGX = 62;   // cells per wave whose L is written (64 lanes, one halo cell each side)
constexpr int kGY = 4;    // lines per workgroup (one wave each)

// line index of the line j across the set of nl lines (ghost lines for j < 0
// or j >= nl); sg = -1 where the transverse momentum is mirrored
__device__ __forceinline__ int gauss_line(int j, int nl, int lo, int hi, double& sg) {
    sg = 1.0;
    if (j >= 0 && j < nl) return j;
    if (lo == PP_BC_PERIODIC) return j < 0 ? j + nl : j - nl;   // |offset| <= 2, nl >= 5
    if (j < 0) {
        if (lo == PP_BC_TRANSMISSIVE) return 0;
        sg = -1.0;
        return min(-1 - j, nl - 1);
    }
    if (hi == PP_BC_TRANSMISSIVE) return nl - 1;
    sg = -1.0;
    return max(2 * nl - 1 - j, 0);
}

// One direction: U, L are [4][nl][n] (lines of n cells, plane stride cs) and
// Wf is [8][nl][n] (planes 0-3: U- at each cell's right face, 4-7: U+ at its
// left face).  A wave holds cells i0-1 .. i0+62 of one line: every lane forms
// and limits its cell's nodes, takes the flux of its left face with the
// right-face nodes of the lane before it, and writes L for cells i0 .. i0+61.
template <int NRM>
__global__ void __launch_bounds__(64 * kGY) gauss_dir_kernel(
    const double* __restrict__ Wf, const double* __restrict__ U, double* __restrict__ L, int n,
    int nl, long long cs, int bc_lo, int bc_hi, int tb_lo, int tb_hi, double h, double gamma,
    double w1, double i12, int flux, double eps_cap, const long long* eps_enc, const Scal* scal,
    GaussCoef G, long long* spd_if) {
    constexpr int TN = 3 - NRM;   // transverse momentum component
    if (scal && !scal->active) return;
    const int lane = threadIdx.x & 63;
    const int l = blockIdx.y * kGY + (threadIdx.x >> 6);
    if (l >= nl) return;   // the whole wave
    const bool cyclic = bc_lo == PP_BC_PERIODIC;
    const int i = blockIdx.x * kGX - 1 + lane;   // -1 .. n + 62
    int ci = i;
    if (cyclic) ci = i < 0 ? i + n : (i >= n ? i - n : i);
    const bool has = cyclic ? (i <= n) : (i >= 0 && i < n);   // lane forms nodes of cell ci
    const double eps_rho = fmin(eps_cap, ord_dec(eps_enc[0]));
    const double eps_e = fmin(eps_cap, ord_dec(eps_enc[1]));
    double Nm[3][4], Np[3][4];
    double sif = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) Nm[k][c] = Np[k][c] = (c == 0 || c == 3) ? 1.0 : 0.0;
    if (has) {
        long long row[5];
        double sg[5];
#pragma unroll
        for (int m = 0; m < 5; ++m)
            row[m] = (long long)gauss_line(l - 2 + m, nl, tb_lo, tb_hi, sg[m]) * n + ci;
        double Ub[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            Ub[c] = U[c * cs + (long long)l * n + ci];
            double vm[5], vp[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                const double s = (c == TN) ? sg[m] : 1.0;
                vm[m] = s * Wf[c * cs + row[m]];
                vp[m] = s * Wf[(4 + c) * cs + row[m]];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double am = 0.0, ap = 0.0;
#pragma unroll
                for (int m = 0; m < 5; ++m) {
                    am += G.c[k][m] * vm[m];
                    ap += G.c[k][m] * vp[m];
                }
                Nm[k][c] = am;
                Np[k][c] = ap;
            }
        }
        pp_limit_nodes<4, NRM>(w1, i12, G.g, eps_rho, eps_e, Ub, Nm, Np);
        if (spd_if) {
            // interface-state rule: |u_n|+a over the average and the six
            // limited node states of the cell
            double sp = wave_speed<4, NRM>(gamma, Ub);
#pragma unroll
            for (int k = 0; k < 3; ++k)
                sp = fmax(sp, fmax(wave_speed<4, NRM>(gamma, Nm[k]), wave_speed<4, NRM>(gamma, Np[k])));
            sif = isfinite(sp) ? sp : INFINITY;
        }
    }
    if (spd_if) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sif = fmax(sif, __shfl_xor(sif, o));
        if (lane == 0) atomicMax(spd_if, ord_enc(sif));
    }
    // left face of this lane's cell: the lane before holds the cell to its left
    double Fl[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double Ul[4], Ur[4], F[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            Ul[c] = __shfl_up(Nm[k][c], 1);
            Ur[c] = Np[k][c];
        }
        if (!cyclic && i == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                Ul[c] = (bc_lo == PP_BC_REFLECTIVE && c == NRM) ? -Ur[c] : Ur[c];
        }
        if (!cyclic && i == n) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                Ur[c] = (bc_hi == PP_BC_REFLECTIVE && c == NRM) ? -Ul[c] : Ul[c];
        }
        if (flux == PP_FLUX_LF) lf_flux<4, NRM>(gamma, Ul, Ur, F);
        else hllc_flux<4, NRM>(gamma, Ul, Ur, F);
#pragma unroll
        for (int c = 0; c < 4; ++c) Fl[c] += G.g[k] * F[c];
    }
    double Fr[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) Fr[c] = __shfl_down(Fl[c], 1);
    if (lane >= 1 && lane <= kGX && i < n) {
#pragma unroll
        for (int c = 0; c < 4; ++c) L[c * cs + (long long)l * n + i] = -(Fr[c] - Fl[c]) / h;
    }
}

// Min rho, min e and max wave speeds of a state [NC][ncell] (x-fastest 2D or 1D).
template <int NC>
__global__ void __launch_bounds__(256) reduce_state_kernel(const double* __restrict__ U,
                                                           long long ncell, double gamma,
                                                           long long* eps_out, long long* spd_out) {
    __shared__ double red[4][4];
    double mr = INFINITY, me = INFINITY, sx = 0.0, sy = 0.0;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < ncell; i += 256LL * gridDim.x) {
        double q[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = U[c * ncell + i];
        mr = fmin(mr, q[0]);
        me = fmin(me, spec_e<NC>(q));
        sx = fmax(sx, wave_speed<NC, 1>(gamma, q));
        if constexpr (NC == 4) sy = fmax(sy, wave_speed<NC, 2>(gamma, q));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mr = fmin(mr, __shfl_xor(mr, o));
        me = fmin(me, __shfl_xor(me, o));
        sx = fmax(sx, __shfl_xor(sx, o));
        sy = fmax(sy, __shfl_xor(sy, o));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = mr; red[w][1] = me; red[w][2] = sx; red[w][3] = sy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 4; ++i) {
            mr = fmin(mr, red[i][0]); me = fmin(me, red[i][1]);
            sx = fmax(sx, red[i][2]); sy = fmax(sy, red[i][3]);
        }
        if (eps_out) {
            atomicMin(&eps_out[0], ord_enc(mr));
            atomicMin(&eps_out[1], ord_enc(me));
        }
        if (spd_out) {
            atomicMax(&spd_out[0], ord_enc(sx));
            atomicMax(&spd_out[1], ord_enc(sy));
        }
    }
}

__global__ void init_scal_kernel(Scal* s) {
    for (int i = 0; i < 3; ++i) s->eps[i][0] = s->eps[i][1] = kEncPosInf;
    s->spd[0] = s->spd[1] = kEncZero;
    s->dt = 0.0;
    s->t = 0.0;
    s->steps = 0;
    s->active = 1;
    s->status = 0u;
    s->stepbad = 0u;
    s->restarts = 0;
    s->spdif[0] = s->spdif[1] = kEncZero;
    s->eps3[0] = s->eps3[1] = kEncPosInf;
    s->redo = 0;
    s->halvings = 0;
}

// Start of a step: advance t by the previous dt, pick the new dt from the
// wave speeds of the current state, clip to t_end / step budget, reset the
// reductions this step will fill.
__device__ __forceinline__ void dt_update(Scal* s, int ndim, int rule, double cfl, double dx,
                                          double dy, double t_end, long long steps_max) {
    if (!s->active) return;   // retired run: later calls change nothing
    if (s->redo) {
        // restart rule: the step is tried again from the same state with the
        // dt the verdict halved; t and the step count stay
        s->redo = 0;
    } else {
        if (s->dt > 0.0) {
            s->t += s->dt;
            s->steps += 1;
        }
        const double sx = ord_dec(s->spd[0]), sy = ord_dec(s->spd[1]);
        double dt = 0.0;
        bool go = s->t < t_end && s->steps < steps_max;
        if (rule != PP_DT_PP) {   // (the interface-state rule picks dt in stage 1)
            if (ndim == 1) dt = (rule == PP_DT_H53 ? cfl * pow(dx, 5.0 / 3.0) : cfl * dx) / sx;
            else dt = cfl / (sx / dx + sy / dy);
            if (go && !(dt > 0.0 && isfinite(dt))) {
                s->status |= 1u;   // no usable wave speed: stop the run
                go = false;
            }
            if (go && s->t + dt > t_end) dt = t_end - s->t;
        }
        s->active = go ? 1 : 0;
        s->dt = go ? dt : 0.0;
    }
    s->spd[0] = s->spd[1] = kEncZero;
    s->eps[0][0] = s->eps[0][1] = kEncPosInf;
    s->eps[1][0] = s->eps[1][1] = kEncPosInf;
}

// Run step of a single grid: t and step count of the finished step, the next
// dt (rule of the run) from the reduced wave speeds, or retire the run.
__global__ void dt_kernel(Scal* s, int ndim, int rule, double cfl, double dx, double dy,
                          double t_end, long long steps_max) {
    dt_update(s, ndim, rule, cfl, dx, dy, t_end, steps_max);
}

// 2D interface-state rule, after the sweeps of stage `stage` (the speeds in
// spdif, which are cleared here for the next stage): stage 1 picks the
// step's dt = cfl / (Sx/dx + Sy/dy), clipped to t_end; stages 2 and 3 set
// status bit 2 when dt (Sx/dx + Sy/dy) > w1 (condition (CFL-CD) broken by
// that stage's input).  A dt that is not usable retires the run.
__global__ void dt_pp2d_kernel(Scal* s, int stage, double cfl, double dx, double dy,
                               double t_end, double w1) {
    if (!s->active) return;
    const double sx = ord_dec(s->spdif[0]), sy = ord_dec(s->spdif[1]);
    s->spdif[0] = s->spdif[1] = kEncZero;
    const double rate = sx / dx + sy / dy;
    if (stage == 1) {
        double dt = cfl / rate;
        if (!(dt > 0.0) || !isfinite(dt)) {
            s->status |= 1u;
            s->active = 0;
            s->dt = 0.0;
            return;
        }
        if (s->t + dt > t_end) dt = t_end - s->t;
        s->dt = dt;
    } else if (s->dt * rate > w1) {
        s->status |= 4u;
    }
}

// Restart rule on the host-driven path (2D, and the explicit and
// characteristic reconstructions in 1D).  The stage-3 output of the step
// being tried sits in the stage-1 buffers (both layouts in 2D); it becomes
// the state when no stage output of the step left G.
__global__ void restart_commit_kernel(const Scal* s, const double* __restrict__ srcA,
                                      double* __restrict__ dstA, const double* __restrict__ srcB,
                                      double* __restrict__ dstB, long long m) {
    if (!s->active || s->stepbad != 0u) return;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        dstA[i] = srcA[i];
        if (dstB) dstB[i] = srcB[i];
    }
}

// ... and the verdict on the step, after the commit: kept (2D: the stage-3
// output's epsilons become those of the next stage-1 input), or redone from
// the same state with half the dt, or, after kMaxHalvings halvings or once
// half the dt no longer moves t (a stall), the run stops with the step's
// status bits.
__global__ void restart_verdict_kernel(Scal* s, int ndim) {
    if (!s->active) return;
    const unsigned bad = s->stepbad;
    s->stepbad = 0u;
    if (bad == 0u) {
        if (ndim == 2) {
            s->eps[2][0] = s->eps3[0];
            s->eps[2][1] = s->eps3[1];
        }
        s->halvings = 0;
        return;
    }
    if (s->halvings >= kMaxHalvings || s->t + 0.5 * s->dt == s->t) {
        s->status |= bad;
        s->active = 0;
        s->dt = 0.0;
        return;
    }
    s->dt *= 0.5;
    s->restarts += 1;
    s->halvings += 1;
    s->redo = 1;
}

// Whole 1D run of a single line in one workgroup: up to max_steps SSP-RK3
// steps (3 stage passes each) with the dt update between steps on thread 0.
// The line's state, stage buffers and scalars are written and read by this
// workgroup only, so block barriers order them.  Ends when the run retires
// (t_end, step budget, unusable dt) or after max_steps steps.
struct RunArgs {
    LineArgs st[3];   // the three stages of a step
    int rule;
    double cfl, t_end;
    long long steps_total;
    int max_steps;
};

template <int NC, int NRM, int W, int CPT, bool SEG1, bool MIXED>
__global__ void __launch_bounds__(2 * NC * 64 * W) run1d_kernel(RunArgs R) {
    extern __shared__ double smem[];
    __shared__ unsigned sbad;
    Scal* s = R.st[0].scal;
    for (int it = 0; it < R.max_steps; ++it) {
        if (threadIdx.x == 0)
            dt_update(s, 1, R.rule, R.cfl, R.st[0].h, 0.0, R.t_end, R.steps_total);
        __syncthreads();
        if (!s->active) break;
        // restart rule: the step is tried, and redone from U^n with half the
        // dt while a stage output leaves G; other rules take one attempt
#pragma unroll 1
        for (int attempt = 0;; ++attempt) {
            if (R.rule == PP_DT_RESTART) {
                if (threadIdx.x == 0) {
                    s->stepbad = 0u;
                    s->spd[0] = kEncZero;   // speeds of this attempt's stage-3 output only
                }
                __syncthreads();
            }
            bool live = true;
#pragma unroll 1
            for (int st = 0; st < 3; ++st) {   // one copy of the operator, stage args by index
                // stage arguments re-read from the kernel-argument segment each
                // time (see line_kernel_persistent)
                typedef __attribute__((address_space(4))) const RunArgs KArgs;
                KArgs* rp = (KArgs*)__builtin_amdgcn_kernarg_segment_ptr();
                asm volatile("" : "+s"(rp));
                line_op<NC, NRM, W, CPT, SEG1, MIXED, true>(((const RunArgs*)rp)->st[st], 0, smem);
                __syncthreads();
                if (!s->active) {   // the interface-state rule found no usable dt
                    live = false;
                    break;
                }
            }
            if (!live || R.rule != PP_DT_RESTART) break;
            if (threadIdx.x == 0)
                sbad = __hip_atomic_load(&s->stepbad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            const unsigned bad = sbad;
            if (bad == 0u) {
                // the step stands: the stage-3 output becomes the state
                const LineArgs& a3 = R.st[2];
                const int n = a3.n;
                for (int q = threadIdx.x; q < NC * n; q += blockDim.x) {
                    const int c = q / n, i = q - c * n;
                    a3.commit[(long long)c * a3.cs + i] = a3.out[(long long)c * a3.cs + i];
                }
                __syncthreads();
                break;
            }
            if (threadIdx.x == 0) {
                // last attempt after kMaxHalvings halvings, or once half the
                // step no longer moves t in FP64 (a stall)
                if (attempt >= kMaxHalvings || s->t + 0.5 * s->dt == s->t) {
                    s->status |= bad;
                    s->active = 0;
                    s->dt = 0.0;
                } else {
                    s->dt *= 0.5;
                    s->restarts += 1;
                }
            }
            __syncthreads();
            if (!s->active) break;
        }
        if (!s->active) break;
    }
}

}  // namespace

// ======================================================================= host
struct pp_cweno_ctx {
    pp_cweno_config cfg{};
    hipStream_t stream = nullptr;
    std::string err;
    int nc = 3;
    long long ncell = 0;
    // single-grid scratch
    double *U1 = nullptr, *U2 = nullptr, *UA = nullptr;        // layout A stage buffers
    double *UB = nullptr, *U1B = nullptr, *U2B = nullptr;      // layout B copies (2D)
    double *Lx = nullptr, *LyB = nullptr;                      // 2D operator halves
    double* Wf = nullptr;    // Gauss-node operator: face values [8][ncell] of one sweep
    int run_rule = PP_DT_CFL;  // run in progress (host-driven steps): its time-step rule, cfl, t_end
    double run_cfl = 0.0, run_t_end = 0.0;
    GaussCoef gcoef{};
    Scal* scal = nullptr;
    // batched
    std::vector<int64_t> lengths;
    std::vector<double> dxs;
    std::vector<int> bcs;
    long long total = 0;
    int maxn = 0;
    long long* d_off = nullptr;
    int* d_n = nullptr;
    double* d_h = nullptr;
    int* d_bc = nullptr;
    double* d_dt = nullptr;
    double* d_t = nullptr;
    long long* d_steps = nullptr;
    int* d_order = nullptr;
    int* d_counter = nullptr;
    double* d_dtcopy = nullptr;
    double* d_tune = nullptr;   // autotuner's scratch copy of the packed state
    double* chs = nullptr;      // characteristic reconstruction: block-solve scratch
    unsigned* d_bad = nullptr;  // restart rule: status bits of each problem's step
    int* d_half = nullptr;      // restart rule: halvings of each problem's step
    int n_sm = 0;
    bool batch_started = false;   // a batched run has set the per-problem t and steps
    // batched launch plan: the length-sorted problems are cut into classes
    // (contiguous in d_order, longest first), one persistent launch per class
    // and stage, each with the kernel shape and LDS of its longest problem
    struct LenClass {
        int begin = 0, count = 0, maxn = 0;
        int w = 1;   // waves per tridiagonal system (64 w lanes; rows per lane n / (64 w))
    };
    std::vector<int> order_host;
    int plan = 0;
    int nclass = 0;
    LenClass cls[3];
    // largest dynamic LDS size already granted to each kernel (the attribute
    // call is a driver round trip, not to be paid on every launch)
    std::unordered_map<const void*, size_t> lds_granted;
    // the allocation-free entry point: every 1D line kernel was granted its
    // largest dynamic LDS at set-up, so launches skip the table above
    bool lds_pregranted = false;
    // measurement: event pairs around kernel launches, per class.  Within a
    // run of back-to-back timed launches (chaining) a launch's begin event is
    // the previous launch's end event, so each launch adds one record.
    bool timing = false;
    std::vector<hipEvent_t> ev[3];    // own events: 2 i (begin), 2 i + 1 (end)
    std::vector<hipEvent_t> beg[3];   // begin event used by launch i
    int nev[3] = {0, 0, 0};
    bool chaining = false;
    hipEvent_t chain = nullptr;       // end event of the last launch, if chaining
};

namespace {

thread_local std::string g_init_err;

int fail(pp_cweno_ctx* c, int code, const std::string& m) {
    if (c) c->err = m;
    else g_init_err = m;
    return code;
}

int hip_fail(pp_cweno_ctx* c, hipError_t e, const char* what) {
    return fail(c, PP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, call)                                   \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

constexpr int kMaxTimed = 4096;

// Record the start event of a timed launch of class k (0 x-lines, 1 y-lines,
// 2 combine); returns the slot or -1.
int timed_begin(pp_cweno_ctx* ctx, int k) {
    if (!ctx->timing || ctx->nev[k] >= kMaxTimed) {
        ctx->chain = nullptr;
        return -1;
    }
    const int i = ctx->nev[k];
    while ((int)ctx->ev[k].size() < 2 * (i + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
            ctx->chain = nullptr;
            return -1;
        }
        ctx->ev[k].push_back(e);
    }
    if ((int)ctx->beg[k].size() < i + 1) ctx->beg[k].resize(i + 1);
    ctx->nev[k] = i + 1;
    if (ctx->chaining && ctx->chain) {
        ctx->beg[k][i] = ctx->chain;   // nothing was enqueued since it was recorded
    } else {
        (void)hipEventRecord(ctx->ev[k][2 * i], ctx->stream);
        ctx->beg[k][i] = ctx->ev[k][2 * i];
    }
    return i;
}

void timed_end(pp_cweno_ctx* ctx, int k, int i) {
    if (i < 0) {
        ctx->chain = nullptr;
        return;
    }
    (void)hipEventRecord(ctx->ev[k][2 * i + 1], ctx->stream);
    ctx->chain = ctx->chaining ? ctx->ev[k][2 * i + 1] : nullptr;
}

// Scope of back-to-back timed launches (nothing else enqueued in between).
struct TimedChain {
    pp_cweno_ctx* ctx;
    explicit TimedChain(pp_cweno_ctx* c) : ctx(c) {
        ctx->chaining = true;
        ctx->chain = nullptr;
    }
    ~TimedChain() {
        ctx->chaining = false;
        ctx->chain = nullptr;
    }
};

// Dynamic LDS of the line kernel for lines of up to nmax cells.
template <int NC, int W, bool MIXED, int RECON = PP_RECON_CWENO>
size_t line_lds_bytes(int nmax, int seg_max) {
    constexpr int NS = 2 * NC, LANES = 64 * W, NT = NS * LANES;
    constexpr int SH = (!MIXED && W == 1 && RECON == PP_RECON_CWENO) ? 4 : 5;   // as the kernel's padding
    const long long LP = padn<SH>(nmax + 2 * kNG - 1) + 1;
    const long long a0 = (long long)NC * LP;
    const long long a1 = (W > 1 || !MIXED) ? (long long)NS * 512 : 0;
    const long long a2 = (long long)NS * (padn<SH>(seg_max + 1) + 1);
    long long m = std::max(a0 + a1, a2);
    return (size_t)(m + NT) * sizeof(double);
}

constexpr size_t kLdsBudget = 160 * 1024;

// Let kernel fn use lds bytes of dynamic LDS (once per size increase; the
// attribute call is a driver round trip, not to be paid on every launch).
int grant_lds(pp_cweno_ctx* ctx, const void* fn, size_t lds) {
    if (ctx->lds_pregranted) return PP_OK;
    size_t& granted = ctx->lds_granted[fn];
    if (lds > granted) {
        HIPCHK(ctx, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        granted = lds;
    }
    return PP_OK;
}

template <int NC, int W, int CPT, bool MIXED, int RECON = PP_RECON_CWENO>
int pick_segment(int nmax) {
    constexpr int NT = 2 * NC * 64 * W;
    int seg = nmax;
    while (seg > 64 &&
           (line_lds_bytes<NC, W, MIXED, RECON>(nmax, seg) > kLdsBudget || (seg + NT - 1) / NT > CPT))
        seg = (seg + 1) / 2;
    return seg;
}

// Launch the line kernel for lines of at most nmax cells; picks the
// single-segment variant when the whole line fits the phase-2 staging.
template <int NC, int NRM, int W, int CPT, bool MIXED>
int launch_line_p(pp_cweno_ctx* ctx, LineArgs A, int nmax, bool persistent, int grid) {
    constexpr int NT = 2 * NC * 64 * W;
    const int seg = pick_segment<NC, W, CPT, MIXED>(nmax);
    A.seg_max = seg;
    const size_t lds = line_lds_bytes<NC, W, MIXED>(nmax, seg);
    if (lds > kLdsBudget || (seg + NT - 1) / NT > CPT)
        return fail(ctx, PP_EUNSUPPORTED, "line too long for the on-chip line kernel");
    const void* fn;
    if (persistent) {
        // batched ensembles are 1D: no persistent 2D kernels are built
        if constexpr (NC == 3)
            fn = seg >= nmax ? (const void*)line_kernel_persistent<NC, NRM, W, CPT, true, MIXED>
                             : (const void*)line_kernel_persistent<NC, NRM, W, CPT, false, MIXED>;
        else
            return fail(ctx, PP_EUNSUPPORTED, "persistent launches serve 1D ensembles only");
    } else if (A.spd_if) {
        // 2D sweeps under the interface-state rule (FP64)
        if constexpr (NC == 4 && !MIXED)
            fn = seg >= nmax
                     ? (const void*)line_kernel<NC, NRM, W, CPT, true, false, PP_RECON_CWENO, true>
                     : (const void*)line_kernel<NC, NRM, W, CPT, false, false, PP_RECON_CWENO, true>;
        else
            return fail(ctx, PP_EUNSUPPORTED, "the 2D interface-state rule runs in FP64");
    } else
        fn = seg >= nmax ? (const void*)line_kernel<NC, NRM, W, CPT, true, MIXED>
                         : (const void*)line_kernel<NC, NRM, W, CPT, false, MIXED>;
    {
        const int rg = grant_lds(ctx, fn, lds);
        if (rg) return rg;
    }
    void* args[] = {&A};
    HIPCHK(ctx, hipLaunchKernel(fn, dim3(persistent ? grid : A.nlines), dim3(NT), args, lds,
                                ctx->stream));
    return PP_OK;
}

// One line launch of an explicit comparison scheme (FP64, not persistent).
template <int NC, int NRM, int W, int CPT, int RECON>
int launch_line_explicit(pp_cweno_ctx* ctx, LineArgs A, int nmax) {
    constexpr int NT = 2 * NC * 64 * W;
    const int seg = pick_segment<NC, W, CPT, false, RECON>(nmax);
    A.seg_max = seg;
    const size_t lds = line_lds_bytes<NC, W, false, RECON>(nmax, seg);
    if (lds > kLdsBudget || (seg + NT - 1) / NT > CPT)
        return fail(ctx, PP_EUNSUPPORTED, "line too long for the on-chip line kernel");
    const void* fn = seg >= nmax ? (const void*)line_kernel<NC, NRM, W, CPT, true, false, RECON>
                                 : (const void*)line_kernel<NC, NRM, W, CPT, false, false, RECON>;
    {
        const int rg = grant_lds(ctx, fn, lds);
        if (rg) return rg;
    }
    void* args[] = {&A};
    HIPCHK(ctx, hipLaunchKernel(fn, dim3(A.nlines), dim3(NT), args, lds, ctx->stream));
    return PP_OK;
}

// Persistent launch of the characteristic-wise or an explicit line kernel
// (batched 1D ensembles, FP64): grid workgroups, each (characteristic) with
// its own row scratch.
template <int NC, int NRM, int W, int CPT, int RECON>
int launch_recon_persistent(pp_cweno_ctx* ctx, LineArgs A, int nmax, int grid) {
    constexpr int NT = 2 * NC * 64 * W;
    const int seg = pick_segment<NC, W, CPT, false, RECON>(nmax);
    A.seg_max = seg;
    const size_t lds = line_lds_bytes<NC, W, false, RECON>(nmax, seg);
    if (lds > kLdsBudget || (seg + NT - 1) / NT > CPT)
        return fail(ctx, PP_EUNSUPPORTED, "line too long for the on-chip line kernel");
    if (grid > ctx->n_sm) return fail(ctx, PP_EINVAL, "persistent grid above the scratch slots");
    const void* fn =
        seg >= nmax ? (const void*)line_kernel_persistent<NC, NRM, W, CPT, true, false, RECON>
                    : (const void*)line_kernel_persistent<NC, NRM, W, CPT, false, false, RECON>;
    {
        const int rg = grant_lds(ctx, fn, lds);
        if (rg) return rg;
    }
    void* args[] = {&A};
    HIPCHK(ctx, hipLaunchKernel(fn, dim3(grid), dim3(NT), args, lds, ctx->stream));
    return PP_OK;
}

template <int NC, int NRM, int W, int CPT>
int launch_line(pp_cweno_ctx* ctx, LineArgs A, int nmax, bool persistent, int grid) {
    if (ctx->cfg.recon != PP_RECON_CWENO) {
        // init admits the other reconstructions only in FP64
        if (ctx->cfg.recon == PP_RECON_CHAR) {
            // every line of a sweep, or every workgroup of a persistent
            // launch, has its own scratch (init sized it for nmax cells)
            A.chs = ctx->chs;
            A.chs_side = char_side_len(NC, nmax);
            A.chs_line = char_line_len(NC, nmax);
            if (persistent) {
                if constexpr (NC == 3)
                    return launch_recon_persistent<NC, NRM, W, CPT, PP_RECON_CHAR>(ctx, A, nmax, grid);
                else return fail(ctx, PP_EUNSUPPORTED, "persistent launches serve 1D ensembles only");
            }
            return launch_line_explicit<NC, NRM, W, CPT, PP_RECON_CHAR>(ctx, A, nmax);
        }
        if (persistent) {
            if constexpr (NC == 3)
                return ctx->cfg.recon == PP_RECON_WENOJS
                           ? launch_recon_persistent<NC, NRM, W, CPT, PP_RECON_WENOJS>(ctx, A, nmax, grid)
                           : launch_recon_persistent<NC, NRM, W, CPT, PP_RECON_WENOZ>(ctx, A, nmax, grid);
            else
                return fail(ctx, PP_EUNSUPPORTED, "persistent launches serve 1D ensembles only");
        }
        return ctx->cfg.recon == PP_RECON_WENOJS
                   ? launch_line_explicit<NC, NRM, W, CPT, PP_RECON_WENOJS>(ctx, A, nmax)
                   : launch_line_explicit<NC, NRM, W, CPT, PP_RECON_WENOZ>(ctx, A, nmax);
    }
    if (ctx->cfg.precision == PP_MIXED)
        return launch_line_p<NC, NRM, W, CPT, true>(ctx, A, nmax, persistent, grid);
    return launch_line_p<NC, NRM, W, CPT, false>(ctx, A, nmax, persistent, grid);
}

LineArgs base_args(const pp_cweno_ctx* ctx) {
    LineArgs A{};
    A.gamma = ctx->cfg.gamma;
    A.w1 = ctx->cfg.gl_w1;
    A.i12 = 1.0 / (1.0 - 2.0 * ctx->cfg.gl_w1);
    A.weno_eps = ctx->cfg.weno_eps;
    A.flux = ctx->cfg.flux;
    A.eps_cap = ctx->cfg.pp_eps_cap;
    A.rk_a = 0.0;
    A.rk_b = 1.0;
    A.status = ctx->scal ? &ctx->scal->status : nullptr;
    return A;
}

// 1D single line: L (mode 0) or stage (mode 1).
int launch_1d(pp_cweno_ctx* ctx, const double* Us, const double* U0, double* out, int mode,
              int stage, double ra, double rb, const double* dt_dev, double dt_val, bool run,
              double* dbg_um = nullptr, double* dbg_up = nullptr, double* dbg_flux = nullptr) {
    LineArgs A = base_args(ctx);
    A.U = Us;
    A.U0 = U0;
    A.out = out;
    A.cs = ctx->cfg.nx;
    A.ls = 0;
    A.n = (int)ctx->cfg.nx;
    A.nlines = 1;
    A.bc_lo = ctx->cfg.bc[0];
    A.bc_hi = ctx->cfg.bc[1];
    A.h = ctx->cfg.dx;
    A.mode = mode;
    A.stage = stage;
    A.rk_a = ra;
    A.rk_b = rb;
    A.dt_dev = dt_dev;
    A.dt_val = dt_val;
    A.scal = run ? ctx->scal : nullptr;
    if (run) {   // the run's time-step rule (stage checks, mode 2)
        A.dtrule = ctx->run_rule;
        A.cfl = ctx->run_cfl;
        A.t_end = ctx->run_t_end;
        // restart rule: a stage output's status bits belong to the step tried
        if (ctx->run_rule == PP_DT_RESTART) A.status = &ctx->scal->stepbad;
    }
    A.dbg_um = dbg_um;
    A.dbg_up = dbg_up;
    A.dbg_flux = dbg_flux;
    if (A.n <= 2048) return launch_line<3, 1, 1, 6>(ctx, A, A.n, false, 1);
    return launch_line<3, 1, 2, 3>(ctx, A, A.n, false, 1);
}

// eq. (RK3) stage coefficients (a, b): U_out = a U^n + b (U_s + dt L(U_s))
const double kRK[4][2] = {{0, 0}, {0.0, 1.0}, {0.75, 0.25}, {1.0 / 3.0, 2.0 / 3.0}};

// Device-resident 1D run: one workgroup, up to max_steps steps per launch.
template <int NC, int NRM, int W, int CPT, bool MIXED>
int launch_run1d_p(pp_cweno_ctx* ctx, RunArgs& R) {
    constexpr int NT = 2 * NC * 64 * W;
    const int nmax = R.st[0].n;
    const int seg = pick_segment<NC, W, CPT, MIXED>(nmax);
    for (auto& a : R.st) a.seg_max = seg;
    const size_t lds = line_lds_bytes<NC, W, MIXED>(nmax, seg);
    if (lds > kLdsBudget || (seg + NT - 1) / NT > CPT)
        return fail(ctx, PP_EUNSUPPORTED, "line too long for the on-chip line kernel");
    const void* fn = seg >= nmax ? (const void*)run1d_kernel<NC, NRM, W, CPT, true, MIXED>
                                 : (const void*)run1d_kernel<NC, NRM, W, CPT, false, MIXED>;
    {
        const int rg = grant_lds(ctx, fn, lds);
        if (rg) return rg;
    }
    void* args[] = {&R};
    HIPCHK(ctx, hipLaunchKernel(fn, dim3(1), dim3(NT), args, lds, ctx->stream));
    return PP_OK;
}

int launch_run1d(pp_cweno_ctx* ctx, double* U, int rule, double cfl, double t_end,
                 long long steps_total, int max_steps) {
    RunArgs R;
    R.rule = rule;
    R.cfl = cfl;
    R.t_end = t_end;
    R.steps_total = steps_total;
    R.max_steps = max_steps;
    const bool restart = rule == PP_DT_RESTART;
    const double* Uin[3] = {U, ctx->U1, ctx->U2};
    // restart rule: stage 3 writes U1 (free after stage 2), committed into U
    // only if the step stays in G
    double* Uout[3] = {ctx->U1, ctx->U2, restart ? ctx->U1 : U};
    for (int st = 1; st <= 3; ++st) {
        LineArgs& a = R.st[st - 1];
        a = base_args(ctx);
        a.U = Uin[st - 1];
        a.U0 = U;
        a.out = Uout[st - 1];
        a.cs = ctx->cfg.nx;
        a.ls = 0;
        a.n = (int)ctx->cfg.nx;
        a.nlines = 1;
        a.bc_lo = ctx->cfg.bc[0];
        a.bc_hi = ctx->cfg.bc[1];
        a.h = ctx->cfg.dx;
        a.mode = (rule == PP_DT_PP && st == 1) ? 2 : 1;
        a.stage = st;
        a.rk_a = kRK[st][0];
        a.rk_b = kRK[st][1];
        a.dt_dev = &ctx->scal->dt;
        a.scal = ctx->scal;
        a.dtrule = rule;
        a.cfl = cfl;
        a.t_end = t_end;
        if (restart) {
            a.status = &ctx->scal->stepbad;
            a.commit = U;
        }
    }
    const bool mixed = ctx->cfg.precision == PP_MIXED;
    if (ctx->cfg.nx <= 2048)
        return mixed ? launch_run1d_p<3, 1, 1, 6, true>(ctx, R)
                     : launch_run1d_p<3, 1, 1, 6, false>(ctx, R);
    return mixed ? launch_run1d_p<3, 1, 2, 3, true>(ctx, R) : launch_run1d_p<3, 1, 2, 3, false>(ctx, R);
}

// Gauss-node sweep along one direction (lines of n cells, nl lines): face
// values in ctx->Wf (written by the line kernel in mode 4) to L.
template <int NRM>
int launch_gauss(pp_cweno_ctx* ctx, const double* Us, double* L, int n, int nl, int bc_lo,
                 int bc_hi, int tb_lo, int tb_hi, double h, const long long* eps_enc, bool run,
                 long long* spd_if) {
    if (!eps_enc) return fail(ctx, PP_EINVAL, "the Gauss-node operator needs the grid's epsilons");
    const auto& c = ctx->cfg;
    const dim3 grid((unsigned)((n + kGX - 1) / kGX), (unsigned)((nl + kGY - 1) / kGY));
    hipLaunchKernelGGL(gauss_dir_kernel<NRM>, grid, dim3(64 * kGY), 0, ctx->stream, ctx->Wf, Us, L,
                       n, nl, (long long)c.nx * c.ny, bc_lo, bc_hi, tb_lo, tb_hi, h, c.gamma,
                       c.gl_w1, 1.0 / (1.0 - 2.0 * c.gl_w1), c.flux, c.pp_eps_cap, eps_enc,
                       run ? ctx->scal : nullptr, ctx->gcoef, spd_if);
    HIPCHK(ctx, hipGetLastError());
    return PP_OK;
}

// 2D sweeps of one stage input (Us in layout A and B) into Lx and LyB.
// spd_if (may be NULL): [2] accumulators of the interface-state rule, x and y.
int sweeps_2d(pp_cweno_ctx* ctx, const double* UsA, const double* UsB, const long long* eps_enc,
              bool run, long long* spd_if = nullptr) {
    const auto& c = ctx->cfg;
    const bool gauss = c.fv == PP_FV_GAUSS;
    LineArgs A = base_args(ctx);
    A.mode = gauss ? 4 : 0;
    // the line kernel reduces the interface speeds itself; under the
    // Gauss-node operator the node kernel does
    A.spd_if = (spd_if && !gauss) ? spd_if : nullptr;
    A.eps_enc = eps_enc;
    A.scal = run ? ctx->scal : nullptr;
    A.cs = (long long)c.nx * c.ny;
    // x-lines: rows of the [4][ny][nx] state
    A.U = UsA;
    A.out = gauss ? ctx->Wf : ctx->Lx;
    A.ls = c.nx;
    A.n = (int)c.nx;
    A.nlines = (int)c.ny;
    A.bc_lo = c.bc[0];
    A.bc_hi = c.bc[1];
    A.h = c.dx;
    int slot = timed_begin(ctx, 0);
    int r = launch_line<4, 1, 1, 4>(ctx, A, A.n, false, 0);
    if (!r && gauss)
        r = launch_gauss<1>(ctx, UsA, ctx->Lx, (int)c.nx, (int)c.ny, c.bc[0], c.bc[1], c.bc[2],
                            c.bc[3], c.dx, eps_enc, run, spd_if);
    timed_end(ctx, 0, slot);
    if (r) return r;
    // y-lines: rows of the transposed [4][nx][ny] state
    A.U = UsB;
    A.out = gauss ? ctx->Wf : ctx->LyB;
    A.ls = c.ny;
    A.n = (int)c.ny;
    A.nlines = (int)c.nx;
    A.bc_lo = c.bc[2];
    A.bc_hi = c.bc[3];
    A.h = c.dy;
    if (A.spd_if) A.spd_if = spd_if + 1;
    slot = timed_begin(ctx, 1);
    r = launch_line<4, 2, 1, 4>(ctx, A, A.n, false, 0);
    if (!r && gauss)
        r = launch_gauss<2>(ctx, UsB, ctx->LyB, (int)c.ny, (int)c.nx, c.bc[2], c.bc[3], c.bc[0],
                            c.bc[1], c.dy, eps_enc, run, spd_if ? spd_if + 1 : nullptr);
    timed_end(ctx, 1, slot);
    return r;
}

int combine_2d(pp_cweno_ctx* ctx, const double* UsA, const double* Un, double* Out, double* OutB,
               int mode, double ra, double rb, const double* dt_dev, double dt_val,
               long long* eps_out, long long* spd_out, long long* eps_reset, bool run) {
    const auto& c = ctx->cfg;
    dim3 grid((unsigned)((c.nx + TC - 1) / TC), (unsigned)((c.ny + TC - 1) / TC));
    const int slot = timed_begin(ctx, 2);
    // restart rule: a stage output's status bits belong to the step tried
    unsigned* const stat =
        !ctx->scal ? nullptr
                   : (run && ctx->run_rule == PP_DT_RESTART ? &ctx->scal->stepbad : &ctx->scal->status);
    hipLaunchKernelGGL(combine2d_kernel, grid, dim3(1024), 0, ctx->stream, ctx->Lx, ctx->LyB, UsA,
                       Un, Out, OutB, (int)c.nx, (int)c.ny, mode, ra, rb, dt_dev, dt_val, c.gamma,
                       eps_out, spd_out, eps_reset, run ? ctx->scal : nullptr, stat);
    timed_end(ctx, 2, slot);
    HIPCHK(ctx, hipGetLastError());
    return PP_OK;
}

int transpose_2d(pp_cweno_ctx* ctx, const double* src, double* dst) {
    const auto& c = ctx->cfg;
    dim3 grid((unsigned)((c.nx + TT - 1) / TT), (unsigned)((c.ny + TT - 1) / TT));
    hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, ctx->stream, src, dst, (int)c.nx,
                       (int)c.ny, 4);
    HIPCHK(ctx, hipGetLastError());
    return PP_OK;
}

int reduce_state(pp_cweno_ctx* ctx, const double* U, long long* eps_out, long long* spd_out) {
    const int grid = (int)std::min<long long>((ctx->ncell + 255) / 256, 4096);
    if (ctx->nc == 3)
        hipLaunchKernelGGL(reduce_state_kernel<3>, dim3(grid), dim3(256), 0, ctx->stream, U,
                           ctx->ncell, ctx->cfg.gamma, eps_out, spd_out);
    else
        hipLaunchKernelGGL(reduce_state_kernel<4>, dim3(grid), dim3(256), 0, ctx->stream, U,
                           ctx->ncell, ctx->cfg.gamma, eps_out, spd_out);
    HIPCHK(ctx, hipGetLastError());
    return PP_OK;
}

int reset_scal(pp_cweno_ctx* ctx) {
    hipLaunchKernelGGL(init_scal_kernel, dim3(1), dim3(1), 0, ctx->stream, ctx->scal);
    HIPCHK(ctx, hipGetLastError());
    return PP_OK;
}


// One full SSP-RK3 step on a single grid (U in/out, layout A; for 2D the
// B copy of U must be current in ctx->UB).  run = take dt and the epsilon
// reductions from the device scalars.
// Restart rule, host-driven runs: commit the step tried (U1 -> U, and
// U1B -> UB in 2D) if no stage output left G, then the verdict kernel.
int restart_end(pp_cweno_ctx* ctx, double* U, double* UB) {
    const long long m = (long long)ctx->nc * ctx->ncell;
    const int grid = (int)std::min<long long>((m + 255) / 256, 2048);
    hipLaunchKernelGGL(restart_commit_kernel, dim3(grid), dim3(256), 0, ctx->stream, ctx->scal,
                       ctx->U1, U, UB ? ctx->U1B : nullptr, UB, m);
    HIPCHK(ctx, hipGetLastError());
    hipLaunchKernelGGL(restart_verdict_kernel, dim3(1), dim3(1), 0, ctx->stream, ctx->scal,
                       ctx->cfg.ndim);
    HIPCHK(ctx, hipGetLastError());
    return PP_OK;
}

int step_single(pp_cweno_ctx* ctx, double* U, const double* dt_dev, double dt_val, bool run) {
    const auto& c = ctx->cfg;
    Scal* s = ctx->scal;
    int r;
    if (c.ndim == 1) {
        // a run under the interface-state rule (the explicit and the
        // characteristic reconstructions; the compact one runs in
        // run1d_kernel): stage 1 picks the step's dt (mode 2), stages 2 and 3
        // check their inputs against it
        const bool pp = run && ctx->run_rule == PP_DT_PP;
        // restart rule: the stage-3 output goes to U1 (free by then) and is
        // committed to U if the step stands
        const bool rs = run && ctx->run_rule == PP_DT_RESTART;
        const double* Uin[3] = {U, ctx->U1, ctx->U2};
        double* Uout[3] = {ctx->U1, ctx->U2, rs ? ctx->U1 : U};
        for (int st = 1; st <= 3; ++st) {
            r = launch_1d(ctx, Uin[st - 1], U, Uout[st - 1], (pp && st == 1) ? 2 : 1, st,
                          kRK[st][0], kRK[st][1], dt_dev, dt_val, run);
            if (r) return r;
        }
        if (rs) return restart_end(ctx, U, nullptr);
        return PP_OK;
    }
    // 2D: stage inputs in both layouts.  Epsilon slots: 2 = stage-1 input
    // (written by the previous stage 3 or the initial reduction), 0 = U1,
    // 1 = U2.  Stage 3 combines in place into U (each element is read and
    // written by the same thread only).
    // Restart rule: stage 3 writes U1 (both layouts; free by then) and its
    // epsilons to eps3, stage 1 clears eps3 instead of slot 2 (slot 2 stays
    // the epsilon of U^n for a retry); the verdict then commits or retries.
    const bool rs = run && ctx->run_rule == PP_DT_RESTART;
    const double* inA[3] = {U, ctx->U1, ctx->U2};
    const double* inB[3] = {ctx->UB, ctx->U1B, ctx->U2B};
    double* outA[3] = {ctx->U1, ctx->U2, rs ? ctx->U1 : U};
    double* outB[3] = {ctx->U1B, ctx->U2B, rs ? ctx->U1B : ctx->UB};
    TimedChain chain(ctx);   // x, y, combine of each stage: nine launches in a row
    for (int st = 1; st <= 3; ++st) {
        const int in_slot = (st + 1) % 3;
        const int out_slot = st - 1;
        const bool ifs = run && ctx->run_rule == PP_DT_PP;
        r = sweeps_2d(ctx, inA[st - 1], inB[st - 1], s->eps[in_slot], run, ifs ? s->spdif : nullptr);
        if (r) return r;
        if (ifs) {
            hipLaunchKernelGGL(dt_pp2d_kernel, dim3(1), dim3(1), 0, ctx->stream, s, st,
                               ctx->run_cfl, c.dx, c.dy, ctx->run_t_end, c.gl_w1);
            HIPCHK(ctx, hipGetLastError());
        }
        long long* const eps_out = (rs && st == 3) ? s->eps3 : s->eps[out_slot];
        long long* const eps_reset = st == 1 ? (rs ? s->eps3 : s->eps[2]) : nullptr;
        r = combine_2d(ctx, inA[st - 1], U, outA[st - 1], outB[st - 1], 1, kRK[st][0], kRK[st][1],
                       dt_dev, dt_val, eps_out, st == 3 ? s->spd : nullptr, eps_reset, run);
        if (r) return r;
    }
    if (rs) return restart_end(ctx, U, ctx->UB);
    return PP_OK;
}

constexpr int kNumPlans = 6;

// Launch plan p: the length cut (p % 3: 0 = one class, 1 = split at 2048
// cells, 2 = split at 2048 and 1024 cells) and the kernel shape of the
// classes of lines up to 2048 cells (p / 3: one wave per system, i.e. chunks
// of up to 32 rows, or 16 in the paired FP64 form, with a 64/128-unknown
// separator system; or two waves per system, chunks of up to 16 rows and a
// 128-unknown separator system, half as many resident lines per CU).  Lines
// longer than 2048 cells always take two waves per system.
void set_plan(pp_cweno_ctx* ctx, int p) {
    const int cuts[3][2] = {{0, 0}, {2048, 0}, {2048, 1024}};
    const int cp = p % 3, short_w = 1 + p / 3;
    ctx->plan = p;
    ctx->nclass = 0;
    const int nb = (int)ctx->order_host.size();
    int i = 0;
    for (int c = 0; c < 3 && i < nb; ++c) {
        const int cut = c < 2 ? cuts[cp][c] : 0;   // class c takes lengths > cut
        auto& k = ctx->cls[ctx->nclass];
        k.begin = i;
        k.maxn = (int)ctx->lengths[ctx->order_host[i]];
        k.w = k.maxn > 2048 ? 2 : short_w;
        while (i < nb && ctx->lengths[ctx->order_host[i]] > cut) ++i;
        k.count = i - k.begin;
        if (k.count > 0) ++ctx->nclass;
        if (cut == 0) break;
    }
}

// One SSP-RK3 step of every active problem of a batch: 3 persistent launches
// per length class of the current plan.
// advance: the stage-3 epilogue advances t, step count and dt per problem.
int batch_step_launch(pp_cweno_ctx* ctx, double* Upacked, double* dtl, bool advance, double cfl,
                      double t_end, long long steps_max) {
    LineArgs A = base_args(ctx);
    // the driver's time-step rule; a step of given dt (advance = false)
    // takes the plain stages
    const int rule = advance ? ctx->cfg.batch_rule : PP_DT_CFL;
    const bool restart = rule == PP_DT_RESTART;
    A.dtrule = rule;
    if (restart) {
        A.badline = ctx->d_bad;
        A.halfline = ctx->d_half;
        A.commit = Upacked;
        A.restart_count = (unsigned long long*)&ctx->scal->restarts;
    }
    A.cs = ctx->total;
    A.off = ctx->d_off;
    A.nline = ctx->d_n;
    A.hline = ctx->d_h;
    A.bcline = ctx->d_bc;
    A.dtline = dtl;
    A.tline = ctx->d_t;
    A.stepline = ctx->d_steps;
    A.steps_max = steps_max;
    A.mode = 1;
    A.t_end = t_end;
    A.cfl = cfl;
    const double* Uin[3] = {Upacked, ctx->U1, ctx->U2};
    // restart rule: stage 3 writes U1, copied into the state per problem only
    // if that problem's step stayed in G
    double* Uout[3] = {ctx->U1, ctx->U2, restart ? ctx->U1 : Upacked};
    for (int st = 1; st <= 3; ++st) {
        A.U = Uin[st - 1];
        A.U0 = Upacked;
        A.out = Uout[st - 1];
        A.mode = (rule == PP_DT_PP && st == 1) ? 2 : 1;
        A.stage = (st == 3 && !advance) ? 0 : st;
        A.rk_a = kRK[st][0];
        A.rk_b = kRK[st][1];
        for (int c = 0; c < ctx->nclass; ++c) {
            const auto& k = ctx->cls[c];
            int* counter = ctx->d_counter + 4 * c + st;
            hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, ctx->stream, counter);
            HIPCHK(ctx, hipGetLastError());
            A.counter = counter;
            A.order = ctx->d_order + k.begin;
            A.nlines = k.count;
            const int grid = std::min(k.count, ctx->n_sm);
            int r = k.w == 1 ? launch_line<3, 1, 1, 6>(ctx, A, k.maxn, true, grid)
                             : launch_line<3, 1, 2, 3>(ctx, A, k.maxn, true, grid);
            if (r) return r;
        }
    }
    return PP_OK;
}

bool bc_ok(int b) { return b == PP_BC_PERIODIC || b == PP_BC_TRANSMISSIVE || b == PP_BC_REFLECTIVE; }

// Allocation-free entry point: per device, the address of that device's
// copy of `scratch` and the dynamic-LDS grants of the 1D line kernels, set
// up once (the first call with that device current).
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
double* g_static_base[kMaxDevices] = {};

template <int W, bool MIXED>
size_t lds_1d_max(int n_lo, int n_hi) {
    size_t m = 0;
    for (int n = n_lo; n <= n_hi; ++n) {
        const int seg = pick_segment<3, W, (W == 1 ? 6 : 3), MIXED>(n);
        m = std::max(m, line_lds_bytes<3, W, MIXED>(n, seg));
    }
    return m;
}

int static_scratch(int dev, double** out) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_base[dev]) {
        static_assert(sizeof(Scal) <= kStaticScalSlots * sizeof(double), "scalars overflow");
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, PP_EDEVICE,
                        std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        // the kernels a 1D step can launch (lines of up to 2048 cells: one
        // wave per system; longer: two), each with its largest LDS
        struct K { const void* fn; size_t lds; };
        const size_t l1 = lds_1d_max<1, false>(3, 2048), l1m = lds_1d_max<1, true>(3, 2048);
        const size_t l2 = lds_1d_max<2, false>(2049, kStaticMaxN);
        const size_t l2m = lds_1d_max<2, true>(2049, kStaticMaxN);
        const K ks[] = {
            {(const void*)line_kernel<3, 1, 1, 6, true, false>, l1},
            {(const void*)line_kernel<3, 1, 1, 6, false, false>, l1},
            {(const void*)line_kernel<3, 1, 1, 6, true, true>, l1m},
            {(const void*)line_kernel<3, 1, 1, 6, false, true>, l1m},
            {(const void*)line_kernel<3, 1, 2, 3, true, false>, l2},
            {(const void*)line_kernel<3, 1, 2, 3, false, false>, l2},
            {(const void*)line_kernel<3, 1, 2, 3, true, true>, l2m},
            {(const void*)line_kernel<3, 1, 2, 3, false, true>, l2m},
        };
        for (const K& k : ks) {
            if (k.lds > kLdsBudget) return fail(nullptr, PP_EUNSUPPORTED, "line kernel LDS budget");
            e = hipFuncSetAttribute(k.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)k.lds);
            if (e != hipSuccess)
                return fail(nullptr, PP_EDEVICE,
                            std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
        }
        g_static_base[dev] = (double*)p;
    }
    *out = g_static_base[dev];
    return PP_OK;
}

// Host-side validation of a configuration (PP_OK or the failing code, with
// the message in the init error slot); no device call.
// Coefficients of the Gauss-node operator.  The quartic q whose averages
// over five unit cells (cell m = [m - 2.5, m - 1.5], m = 0..4) are v_m is the
// derivative of the quintic P through the cell edges x_e = e - 2.5 with
// P(x_e) = v_0 + ... + v_{e-1}; so q(xi) = sum_m v_m sum_{e > m} l_e'(xi) with
// l_e the Lagrange basis on the edges.  Nodes: the three Gauss-Legendre
// points of the middle cell; weights 5/18, 8/18, 5/18.
GaussCoef gauss_coef() {
    GaussCoef G{};
    const double xi[3] = {-std::sqrt(15.0) / 10.0, 0.0, std::sqrt(15.0) / 10.0};
    double xe[6];
    for (int e = 0; e < 6; ++e) xe[e] = e - 2.5;
    for (int k = 0; k < 3; ++k) {
        double dl[6];   // l_e'(xi_k)
        for (int e = 0; e < 6; ++e) {
            double le = 1.0, sum = 0.0;
            for (int j = 0; j < 6; ++j) {
                if (j == e) continue;
                le *= (xi[k] - xe[j]) / (xe[e] - xe[j]);
                sum += 1.0 / (xi[k] - xe[j]);
            }
            dl[e] = le * sum;
        }
        for (int m = 0; m < 5; ++m) {
            double a = 0.0;
            for (int e = m + 1; e < 6; ++e) a += dl[e];
            G.c[k][m] = a;
        }
    }
    G.g[0] = G.g[2] = 5.0 / 18.0;
    G.g[1] = 8.0 / 18.0;
    return G;
}

int check_config(const pp_cweno_config& c) {
    if (c.ndim != 1 && c.ndim != 2) return fail(nullptr, PP_EINVAL, "ndim must be 1 or 2");
    if (!(c.gamma > 1.0)) return fail(nullptr, PP_EINVAL, "gamma must be > 1");
    if (!(c.gl_w1 > 0.0 && c.gl_w1 < 0.5)) return fail(nullptr, PP_EINVAL, "gl_w1 must be in (0, 1/2)");
    if (c.flux != PP_FLUX_HLLC && c.flux != PP_FLUX_LF)
        return fail(nullptr, PP_EINVAL, "flux must be PP_FLUX_HLLC or PP_FLUX_LF");
    if (c.recon != PP_RECON_CWENO && c.recon != PP_RECON_WENOJS && c.recon != PP_RECON_WENOZ &&
        c.recon != PP_RECON_CHAR)
        return fail(nullptr, PP_EINVAL, "recon must be PP_RECON_CWENO, _WENOJS, _WENOZ or _CHAR");
    if (c.recon != PP_RECON_CWENO && c.precision != PP_FP64)
        return fail(nullptr, PP_EUNSUPPORTED, "the explicit and characteristic schemes run in FP64");
    if (!(c.weno_eps > 0.0) || !(c.pp_eps_cap > 0.0))
        return fail(nullptr, PP_EINVAL, "epsilons must be > 0");
    if (c.precision != PP_FP64 && c.precision != PP_MIXED)
        return fail(nullptr, PP_EINVAL, "precision must be PP_FP64 or PP_MIXED");
    if (c.batch_rule != PP_DT_CFL && c.batch_rule != PP_DT_PP && c.batch_rule != PP_DT_RESTART)
        return fail(nullptr, PP_EINVAL, "batch_rule must be PP_DT_CFL, PP_DT_PP or PP_DT_RESTART");
    if (c.fv != PP_FV_LINE && c.fv != PP_FV_GAUSS)
        return fail(nullptr, PP_EINVAL, "fv must be PP_FV_LINE or PP_FV_GAUSS");
    if (c.fv == PP_FV_GAUSS &&
        (c.ndim != 2 || c.precision != PP_FP64 || c.recon != PP_RECON_CWENO || c.nbatch > 0))
        return fail(nullptr, PP_EUNSUPPORTED,
                    "the Gauss-node operator is 2D, FP64 and the compact reconstruction");
    const int naxes = c.ndim == 2 ? 2 : 1;
    for (int a = 0; a < naxes; ++a) {
        if (!bc_ok(c.bc[2 * a]) || !bc_ok(c.bc[2 * a + 1]))
            return fail(nullptr, PP_EINVAL, "unknown boundary code");
        if ((c.bc[2 * a] == PP_BC_PERIODIC) != (c.bc[2 * a + 1] == PP_BC_PERIODIC))
            return fail(nullptr, PP_EINVAL, "periodic must be set on both ends of an axis");
    }
    if (c.nbatch < 0) return fail(nullptr, PP_EINVAL, "nbatch < 0");
    if (c.nbatch > 0) {
        if (c.ndim != 1) return fail(nullptr, PP_EINVAL, "batched ensembles are 1D");
        if (!c.lengths || !c.dxs || !c.bcs) return fail(nullptr, PP_EINVAL, "batch arrays are NULL");
        for (int64_t i = 0; i < c.nbatch; ++i) {
            if (c.lengths[i] < 3) return fail(nullptr, PP_EINVAL, "batched problem with < 3 cells");
            if (c.lengths[i] > 4096) return fail(nullptr, PP_EUNSUPPORTED, "batched problem > 4096 cells");
            if (!(c.dxs[i] > 0.0)) return fail(nullptr, PP_EINVAL, "batched dx must be > 0");
            for (int e = 0; e < 2; ++e)
                if (!bc_ok(c.bcs[2 * i + e]) || c.bcs[2 * i + e] == PP_BC_PERIODIC)
                    return fail(nullptr, PP_EINVAL, "batched problems need non-periodic codes");
        }
    } else {
        const int64_t nmin_x = c.bc[0] == PP_BC_PERIODIC ? 5 : 3;
        if (c.nx < nmin_x) return fail(nullptr, PP_EINVAL, "nx too small");
        if (!(c.dx > 0.0)) return fail(nullptr, PP_EINVAL, "dx must be > 0");
        if (c.ndim == 1) {
            if (c.nx > 4096) return fail(nullptr, PP_EUNSUPPORTED, "1D lines are limited to 4096 cells");
        } else {
            const int64_t nmin_y = c.bc[2] == PP_BC_PERIODIC ? 5 : 3;
            if (c.ny < nmin_y) return fail(nullptr, PP_EINVAL, "ny too small");
            if (!(c.dy > 0.0)) return fail(nullptr, PP_EINVAL, "dy must be > 0");
            if (c.nx > 2048 || c.ny > 2048)
                return fail(nullptr, PP_EUNSUPPORTED, "2D lines are limited to 2048 cells");
        }
    }
    return PP_OK;
}

}  // namespace

extern "C" {

void pp_cweno_config_defaults(pp_cweno_config* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->ndim = 1;
    cfg->ny = 1;
    cfg->gamma = 1.4;
    cfg->weno_eps = 1e-13;
    cfg->pp_eps_cap = 1e-13;
    cfg->gl_w1 = 1.0 / 12.0;
    cfg->precision = PP_FP64;
}

int pp_cweno_init(const pp_cweno_config* cfg, pp_cweno_ctx** out) {
    if (!out) return fail(nullptr, PP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(nullptr, PP_EINVAL, "cfg is NULL");
    const pp_cweno_config& c = *cfg;
    const int v = check_config(c);
    if (v) return v;
    auto* ctx = new (std::nothrow) pp_cweno_ctx();
    if (!ctx) return fail(nullptr, PP_ENOMEM, "host allocation failed");
    ctx->cfg = c;
    ctx->cfg.lengths = nullptr;
    ctx->cfg.dxs = nullptr;
    ctx->cfg.bcs = nullptr;
    ctx->stream = (hipStream_t)c.stream;
    ctx->nc = c.ndim == 2 ? 4 : 3;
    auto bail = [&](int code) {
        g_init_err = ctx->err;
        pp_cweno_destroy(ctx);
        return code;
    };
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        hip_fail(ctx, e, "hipGetDevice");
        return bail(PP_EDEVICE);
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ctx->n_sm = prop.multiProcessorCount;
    if (ctx->n_sm <= 0) ctx->n_sm = 256;
    auto dmalloc = [&](void** p, size_t bytes) -> bool {
        hipError_t er = hipMalloc(p, bytes);
        if (er != hipSuccess) {
            hip_fail(ctx, er, "hipMalloc");
            return false;
        }
        return true;
    };
    if (!dmalloc((void**)&ctx->scal, sizeof(Scal))) return bail(PP_ENOMEM);
    if (c.nbatch > 0) {
        const int64_t nb = c.nbatch;
        ctx->lengths.assign(c.lengths, c.lengths + nb);
        ctx->dxs.assign(c.dxs, c.dxs + nb);
        ctx->bcs.assign(c.bcs, c.bcs + 2 * nb);
        std::vector<long long> off(nb + 1, 0);
        for (int64_t i = 0; i < nb; ++i) {
            off[i + 1] = off[i] + c.lengths[i];
            ctx->maxn = std::max<int>(ctx->maxn, (int)c.lengths[i]);
        }
        ctx->total = off[nb];
        ctx->ncell = ctx->total;
        // characteristic reconstruction: row scratch per workgroup slot of the
        // persistent launches (at most one workgroup per CU per launch)
        if (c.recon == PP_RECON_CHAR &&
            !dmalloc((void**)&ctx->chs, sizeof(double) * (size_t)ctx->n_sm * (size_t)char_line_len(3, ctx->maxn)))
            return bail(PP_ENOMEM);
        std::vector<int> order(nb), ln(nb);
        for (int64_t i = 0; i < nb; ++i) {
            order[i] = (int)i;
            ln[i] = (int)c.lengths[i];
        }
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return ln[a] > ln[b]; });
        if (!dmalloc((void**)&ctx->d_off, sizeof(long long) * (nb + 1)) ||
            !dmalloc((void**)&ctx->d_n, sizeof(int) * nb) ||
            !dmalloc((void**)&ctx->d_h, sizeof(double) * nb) ||
            !dmalloc((void**)&ctx->d_bc, sizeof(int) * 2 * nb) ||
            !dmalloc((void**)&ctx->d_dt, sizeof(double) * nb) ||
            !dmalloc((void**)&ctx->d_dtcopy, sizeof(double) * nb) ||
            !dmalloc((void**)&ctx->d_t, sizeof(double) * nb) ||
            !dmalloc((void**)&ctx->d_steps, sizeof(long long) * nb) ||
            !dmalloc((void**)&ctx->d_order, sizeof(int) * nb) ||
            !dmalloc((void**)&ctx->d_counter, sizeof(int) * 16) ||
            !dmalloc((void**)&ctx->d_bad, sizeof(unsigned) * nb) ||
            !dmalloc((void**)&ctx->d_half, sizeof(int) * nb) ||
            !dmalloc((void**)&ctx->U1, sizeof(double) * 3 * ctx->total) ||
            !dmalloc((void**)&ctx->U2, sizeof(double) * 3 * ctx->total))
            return bail(PP_ENOMEM);
        hipError_t e2 = hipSuccess;
        e2 = e2 == hipSuccess ? hipMemcpy(ctx->d_off, off.data(), sizeof(long long) * (nb + 1), hipMemcpyHostToDevice) : e2;
        e2 = e2 == hipSuccess ? hipMemcpy(ctx->d_n, ln.data(), sizeof(int) * nb, hipMemcpyHostToDevice) : e2;
        e2 = e2 == hipSuccess ? hipMemcpy(ctx->d_h, c.dxs, sizeof(double) * nb, hipMemcpyHostToDevice) : e2;
        e2 = e2 == hipSuccess ? hipMemcpy(ctx->d_bc, c.bcs, sizeof(int) * 2 * nb, hipMemcpyHostToDevice) : e2;
        e2 = e2 == hipSuccess ? hipMemcpy(ctx->d_order, order.data(), sizeof(int) * nb, hipMemcpyHostToDevice) : e2;
        if (e2 != hipSuccess) {
            hip_fail(ctx, e2, "hipMemcpy");
            return bail(PP_EDEVICE);
        }
        ctx->order_host = order;
        set_plan(ctx, 0);
    } else {
        ctx->ncell = c.nx * (c.ndim == 2 ? c.ny : 1);
        const size_t bytes = sizeof(double) * ctx->nc * ctx->ncell;
        if (!dmalloc((void**)&ctx->U1, bytes) || !dmalloc((void**)&ctx->U2, bytes))
            return bail(PP_ENOMEM);
        if (c.recon == PP_RECON_CHAR) {
            // the block-solve scratch of every line of a sweep (2D: the
            // larger of the x sweep's ny lines and the y sweep's nx lines)
            const long long len = c.ndim == 2
                                      ? std::max((long long)c.ny * char_line_len(4, (int)c.nx),
                                                 (long long)c.nx * char_line_len(4, (int)c.ny))
                                      : char_line_len(3, (int)c.nx);
            if (!dmalloc((void**)&ctx->chs, sizeof(double) * (size_t)len)) return bail(PP_ENOMEM);
        }
        if (c.ndim == 2) {
            if (!dmalloc((void**)&ctx->UA, bytes) || !dmalloc((void**)&ctx->UB, bytes) ||
                !dmalloc((void**)&ctx->U1B, bytes) || !dmalloc((void**)&ctx->U2B, bytes) ||
                !dmalloc((void**)&ctx->Lx, bytes) || !dmalloc((void**)&ctx->LyB, bytes))
                return bail(PP_ENOMEM);
            if (c.fv == PP_FV_GAUSS) {
                if (!dmalloc((void**)&ctx->Wf, 2 * bytes)) return bail(PP_ENOMEM);
                ctx->gcoef = gauss_coef();
            }
        }
    }
    if (reset_scal(ctx)) return bail(PP_EDEVICE);
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        hip_fail(ctx, e, "hipStreamSynchronize");
        return bail(PP_EDEVICE);
    }
    *out = ctx;
    return PP_OK;
}

int pp_cweno_rhs(pp_cweno_ctx* ctx, const double* U, double* L) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    if (!U || !L) return fail(ctx, PP_EINVAL, "U or L is NULL");
    if (U == L) return fail(ctx, PP_EINVAL, "U and L must be distinct");
    if (ctx->cfg.nbatch > 0) return fail(ctx, PP_EINVAL, "pp_cweno_rhs needs a single grid");
    if (ctx->cfg.ndim == 1) return launch_1d(ctx, U, nullptr, L, 0, 0, 0.0, 1.0, nullptr, 0.0, false);
    // 2D: epsilon of U into slot 0 of the scalars, transposed copy, sweeps, sum
    int r = reset_scal(ctx);
    if (!r) r = reduce_state(ctx, U, ctx->scal->eps[0], nullptr);
    if (!r) r = transpose_2d(ctx, U, ctx->UB);
    if (!r) r = sweeps_2d(ctx, U, ctx->UB, ctx->scal->eps[0], false);
    if (!r) r = combine_2d(ctx, U, nullptr, L, nullptr, 0, 0.0, 1.0, nullptr, 0.0, nullptr, nullptr,
                           nullptr, false);
    return r;
}

int pp_cweno_stage(pp_cweno_ctx* ctx, const double* U0, const double* Us, double* Uout, int stage,
                   double dt) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    if (!U0 || !Us || !Uout) return fail(ctx, PP_EINVAL, "NULL state pointer");
    if (Uout == U0 || Uout == Us) return fail(ctx, PP_EINVAL, "Uout must not alias U0 or Us");
    if (stage < 1 || stage > 3) return fail(ctx, PP_EINVAL, "stage must be 1, 2 or 3");
    if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(ctx, PP_EINVAL, "dt must be finite and >= 0");
    if (ctx->cfg.nbatch > 0) return fail(ctx, PP_EINVAL, "pp_cweno_stage needs a single grid");
    if (ctx->cfg.ndim == 1)
        return launch_1d(ctx, Us, U0, Uout, 1, stage, kRK[stage][0], kRK[stage][1], nullptr, dt, false);
    int r = reset_scal(ctx);
    if (!r) r = reduce_state(ctx, Us, ctx->scal->eps[0], nullptr);
    if (!r) r = transpose_2d(ctx, Us, ctx->U1B);
    if (!r) r = sweeps_2d(ctx, Us, ctx->U1B, ctx->scal->eps[0], false);
    if (!r) r = combine_2d(ctx, Us, U0, Uout, ctx->U2B, 1, kRK[stage][0], kRK[stage][1], nullptr, dt,
                           ctx->scal->eps[1], nullptr, nullptr, false);
    return r;
}

int pp_cweno_step(pp_cweno_ctx* ctx, double* U, double dt) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    if (!U) return fail(ctx, PP_EINVAL, "U is NULL");
    if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(ctx, PP_EINVAL, "dt must be finite and >= 0");
    if (ctx->cfg.nbatch > 0) return fail(ctx, PP_EINVAL, "use pp_cweno_batch_step for ensembles");
    int r = reset_scal(ctx);
    if (r) return r;
    if (ctx->cfg.ndim == 2) {
        r = reduce_state(ctx, U, ctx->scal->eps[2], nullptr);
        if (!r) r = transpose_2d(ctx, U, ctx->UB);
        if (r) return r;
    }
    return step_single(ctx, U, nullptr, dt, false);
}

int pp_cweno_step_static(const pp_cweno_config* cfg, double* U, double dt) {
    if (!cfg || !U) return fail(nullptr, PP_EINVAL, "cfg or U is NULL");
    const pp_cweno_config& c = *cfg;
    const int v = check_config(c);
    if (v) return v;
    if (c.ndim != 1 || c.nbatch != 0)
        return fail(nullptr, PP_EINVAL, "pp_cweno_step_static advances one 1D line");
    if (c.recon != PP_RECON_CWENO)
        return fail(nullptr, PP_EUNSUPPORTED, "pp_cweno_step_static runs the compact scheme");
    if (c.nx > kStaticMaxN)
        return fail(nullptr, PP_EUNSUPPORTED, "pp_cweno_step_static: at most 4096 cells");
    if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(nullptr, PP_EINVAL, "dt must be finite and >= 0");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, PP_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(nullptr, PP_EUNSUPPORTED, "device index beyond the static scratch table");
    double* base = nullptr;
    int r = static_scratch(dev, &base);
    if (r) return r;
    // launch state on the stack; device memory is the scratch array only
    pp_cweno_ctx ctx;
    ctx.cfg = c;
    ctx.cfg.lengths = nullptr;
    ctx.cfg.dxs = nullptr;
    ctx.cfg.bcs = nullptr;
    ctx.stream = (hipStream_t)c.stream;
    ctx.nc = 3;
    ctx.ncell = c.nx;
    ctx.scal = reinterpret_cast<Scal*>(base);
    ctx.U1 = base + kStaticScalSlots;
    ctx.U2 = ctx.U1 + 3 * kStaticMaxN;
    ctx.lds_pregranted = true;
    r = reset_scal(&ctx);   // clears the scalars the last call left
    if (!r) r = step_single(&ctx, U, nullptr, dt, false);
    if (r) g_init_err = ctx.err;
    return r;
}

int pp_cweno_run(pp_cweno_ctx* ctx, double* U, double t_end, int64_t nsteps_max, double cfl,
                 int rule, double* t_out, int64_t* steps_out) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    if (!U) return fail(ctx, PP_EINVAL, "U is NULL");
    if (!(t_end > 0.0) || !(cfl > 0.0) || nsteps_max < 0)
        return fail(ctx, PP_EINVAL, "t_end and cfl must be > 0, nsteps_max >= 0");
    if (rule != PP_DT_CFL && rule != PP_DT_H53 && rule != PP_DT_PP && rule != PP_DT_RESTART)
        return fail(ctx, PP_EINVAL, "unknown dt rule");
    if (rule == PP_DT_H53 && ctx->cfg.ndim != 1) return fail(ctx, PP_EINVAL, "h^(5/3) rule is 1D");
    if (ctx->cfg.nbatch > 0) return fail(ctx, PP_EINVAL, "use pp_cweno_batch_run for ensembles");
    if (rule == PP_DT_PP && ctx->cfg.ndim == 2 && ctx->cfg.precision != PP_FP64)
        return fail(ctx, PP_EUNSUPPORTED, "the 2D interface-state rule runs in FP64");
    const auto& c = ctx->cfg;
    Scal* s = ctx->scal;
    int r = reset_scal(ctx);
    if (!r) r = reduce_state(ctx, U, s->eps[2], s->spd);
    if (!r && c.ndim == 2) r = transpose_2d(ctx, U, ctx->UB);
    if (r) return r;
    Scal host{};
    if (c.ndim == 1 && c.recon == PP_RECON_CWENO) {
        // one workgroup runs the line for up to 4096 steps per launch; the
        // host checks the scalars between launches
        for (;;) {
            r = launch_run1d(ctx, U, rule, cfl, t_end, (long long)nsteps_max, 4096);
            if (r) return r;
            HIPCHK(ctx, hipMemcpyAsync(&host, s, sizeof(Scal), hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            if (!host.active) break;
        }
        if (t_out) *t_out = host.t;
        if (steps_out) *steps_out = host.steps;
        if (host.status & 3u)
            return fail(ctx, PP_ESTATE, "a stage left the admissible set or was not finite");
        return PP_OK;
    }
    // 2D, and the explicit and characteristic schemes in 1D: (dt kernel,
    // step) pairs, launched in groups (below); the dt kernel retires the run
    // at t_end or after nsteps_max steps (later launches return at once),
    // and each group ends with a host check of the scalars.  Under the 2D
    // interface-state rule each stage's sweeps also reduce the interface
    // speeds and a small kernel picks (stage 1) or checks (stages 2 and 3)
    // the dt before the stage's combine; under the restart rule each step
    // ends with its commit and verdict kernels.
    struct RunRule {
        pp_cweno_ctx* ctx;
        ~RunRule() { ctx->run_rule = PP_DT_CFL; }
    } rule_guard{ctx};
    ctx->run_rule = rule;
    ctx->run_cfl = cfl;
    ctx->run_t_end = t_end;
    auto launch_group = [&](int64_t count) -> int {
        for (int64_t i = 0; i < count; ++i) {
            hipLaunchKernelGGL(dt_kernel, dim3(1), dim3(1), 0, ctx->stream, s, c.ndim, rule, cfl,
                               c.dx, c.dy, t_end, (long long)nsteps_max);
            HIPCHK(ctx, hipGetLastError());
            const int rs = step_single(ctx, U, &s->dt, 0.0, true);
            if (rs) return rs;
        }
        return PP_OK;
    };
    auto check = [&](hipStream_t st) -> int {
        HIPCHK(ctx, hipMemcpyAsync(&host, s, sizeof(Scal), hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        return PP_OK;
    };
    // The first group runs eagerly (it also sets the kernels' LDS limits).
    // Later groups replay one captured group: a hipGraph of kRunGroup
    // (dt kernel, step) pairs on a private stream ordered after the
    // caller's, so a long run of small grids is not bound by launch
    // overhead.  With kernel timing on, every group is launched eagerly.
    constexpr int64_t kRunGroup = 16;
    int64_t launched = std::max<int64_t>(1, std::min<int64_t>(kRunGroup, nsteps_max + 1));
    r = launch_group(launched);
    if (!r) r = check(ctx->stream);
    if (r) return r;
    if (host.active && ctx->timing) {
        for (;;) {
            const int64_t batch = std::max<int64_t>(1, std::min<int64_t>(64, nsteps_max - launched + 1));
            r = launch_group(batch);
            if (!r) r = check(ctx->stream);
            if (r) return r;
            launched += batch;
            if (!host.active) break;
        }
    } else if (host.active) {
        hipStream_t user = ctx->stream, gs = nullptr;
        hipEvent_t ev = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        auto cleanup = [&]() {
            ctx->stream = user;
            if (gs) (void)hipStreamSynchronize(gs);
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            if (ev) (void)hipEventDestroy(ev);
            if (gs) (void)hipStreamDestroy(gs);
        };
        hipError_t e = hipStreamCreateWithFlags(&gs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev, user);
        if (e == hipSuccess) e = hipStreamWaitEvent(gs, ev, 0);
        if (e == hipSuccess) e = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            cleanup();
            return hip_fail(ctx, e, "run graph capture");
        }
        ctx->stream = gs;
        r = launch_group(kRunGroup);
        e = hipStreamEndCapture(gs, &graph);
        ctx->stream = user;
        if (!r && e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (r || e != hipSuccess) {
            cleanup();
            return r ? r : hip_fail(ctx, e, "run graph capture");
        }
        // the dt kernel retires the run at t_end or nsteps_max; the pairs of a
        // replay after that return at once
        for (;;) {
            e = hipGraphLaunch(exec, gs);
            if (e == hipSuccess) e = hipMemcpyAsync(&host, s, sizeof(Scal), hipMemcpyDeviceToHost, gs);
            if (e == hipSuccess) e = hipStreamSynchronize(gs);
            if (e != hipSuccess) {
                cleanup();
                return hip_fail(ctx, e, "run graph replay");
            }
            if (!host.active) break;
        }
        cleanup();
    }
    if (t_out) *t_out = host.t;
    if (steps_out) *steps_out = host.steps;
    if (host.status & 3u)
        return fail(ctx, PP_ESTATE, "a stage left the admissible set or was not finite");
    return PP_OK;
}

int pp_cweno_restarts(pp_cweno_ctx* ctx, int64_t* out) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    if (!out) return fail(ctx, PP_EINVAL, "out is NULL");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    long long v = 0;
    HIPCHK(ctx, hipMemcpy(&v, &ctx->scal->restarts, sizeof(v), hipMemcpyDeviceToHost));
    *out = v;
    return PP_OK;
}

int pp_cweno_max_speed(pp_cweno_ctx* ctx, const double* U, double* out_dev) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    if (!U || !out_dev) return fail(ctx, PP_EINVAL, "NULL pointer");
    int r = reset_scal(ctx);
    if (!r) r = reduce_state(ctx, U, nullptr, ctx->scal->spd);
    if (r) return r;
    // decode on the device side through a tiny copy of the encoded values
    long long enc[2];
    HIPCHK(ctx, hipMemcpyAsync(enc, ctx->scal->spd, sizeof(enc), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    double v[2];
    for (int i = 0; i < 2; ++i) {
        long long x = enc[i] >= 0 ? enc[i] : (enc[i] ^ 0x7fffffffffffffffLL);
        std::memcpy(&v[i], &x, sizeof(double));
    }
    HIPCHK(ctx, hipMemcpyAsync(out_dev, v, sizeof(double) * (ctx->cfg.ndim == 2 ? 2 : 1),
                               hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return PP_OK;
}

int pp_cweno_batch_step(pp_cweno_ctx* ctx, double* Upacked, const double* dt_dev) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    if (!Upacked || !dt_dev) return fail(ctx, PP_EINVAL, "NULL pointer");
    if (ctx->cfg.nbatch <= 0) return fail(ctx, PP_EINVAL, "context has no batch");
    // the kernels read each problem's dt from a private copy so the caller's
    // array stays read-only
    HIPCHK(ctx, hipMemcpyAsync(ctx->d_dtcopy, dt_dev, sizeof(double) * ctx->cfg.nbatch,
                               hipMemcpyDeviceToDevice, ctx->stream));
    return batch_step_launch(ctx, Upacked, ctx->d_dtcopy, false, 0.0, 0.0, 0);
}

int pp_cweno_batch_tune(pp_cweno_ctx* ctx, const double* Upacked, double cfl, int force_plan,
                        int* plan_out, double* ms_out) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    if (ctx->cfg.nbatch <= 0) return fail(ctx, PP_EINVAL, "context has no batch");
    if (force_plan >= kNumPlans) return fail(ctx, PP_EINVAL, "unknown launch plan");
    if (force_plan >= 0) {
        set_plan(ctx, force_plan);
        if (plan_out) *plan_out = force_plan;
        return PP_OK;
    }
    if (!Upacked) return fail(ctx, PP_EINVAL, "Upacked is NULL");
    if (!(cfl > 0.0)) return fail(ctx, PP_EINVAL, "cfl must be > 0");
    const int nb = (int)ctx->cfg.nbatch;
    const size_t bytes = sizeof(double) * 3 * ctx->total;
    if (!ctx->d_tune && hipMalloc((void**)&ctx->d_tune, bytes) != hipSuccess) {
        ctx->d_tune = nullptr;
        return fail(ctx, PP_ENOMEM, "autotuner scratch");
    }
    // per-problem dt of the initial state (the run's first step); this
    // overwrites the per-problem t and steps, so no run can be continued
    hipLaunchKernelGGL(batch_init_kernel, dim3(nb), dim3(256), 0, ctx->stream, Upacked, ctx->total,
                       ctx->d_off, ctx->d_n, ctx->d_h, ctx->d_dt, ctx->d_t, ctx->d_steps,
                       ctx->cfg.gamma, cfl, 1e300, 0, 0LL, PP_DT_CFL, nullptr, nullptr);
    ctx->batch_started = false;
    HIPCHK(ctx, hipGetLastError());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, PP_EDEVICE, "hipEventCreate");
    }
    const int reps = 3;
    int best = -1;
    float best_ms = 0.0f;
    int r = PP_OK;
    for (int p = 0; p < kNumPlans && r == PP_OK; ++p) {
        set_plan(ctx, p);
        float ms = -1.0f;
        // one warm-up step, then reps timed steps of the same state and dt
        for (int it = 0; it <= reps && r == PP_OK; ++it) {
            if (hipMemcpyAsync(ctx->d_tune, Upacked, bytes, hipMemcpyDeviceToDevice, ctx->stream) !=
                    hipSuccess ||
                hipMemcpyAsync(ctx->d_dtcopy, ctx->d_dt, sizeof(double) * nb,
                               hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess) {
                r = fail(ctx, PP_EDEVICE, "autotuner copy");
                break;
            }
            if (it == 1) (void)hipEventRecord(e0, ctx->stream);
            r = batch_step_launch(ctx, ctx->d_tune, ctx->d_dtcopy, false, 0.0, 0.0, 0);
        }
        if (r) break;
        (void)hipEventRecord(e1, ctx->stream);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            r = fail(ctx, PP_EDEVICE, "autotuner timing");
            break;
        }
        ms /= reps;   // includes the two state copies of each repetition
        if (ms_out) ms_out[p] = ms;
        if (best < 0 || ms < best_ms) {
            best = p;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r) return r;
    set_plan(ctx, best);
    if (plan_out) *plan_out = best;
    return PP_OK;
}

static int batch_run_impl(pp_cweno_ctx* ctx, double* Upacked, double t_end, int64_t nsteps_max,
                          double cfl, int64_t* steps_out, double* t_out, bool resume) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    if (!Upacked) return fail(ctx, PP_EINVAL, "Upacked is NULL");
    if (ctx->cfg.nbatch <= 0) return fail(ctx, PP_EINVAL, "context has no batch");
    if (!(t_end > 0.0) || !(cfl > 0.0) || nsteps_max < 1)
        return fail(ctx, PP_EINVAL, "t_end and cfl must be > 0, nsteps_max >= 1");
    if (resume && !ctx->batch_started)
        return fail(ctx, PP_EINVAL, "pp_cweno_batch_continue needs a pp_cweno_batch_run first");
    const int nb = (int)ctx->cfg.nbatch;
    int r = 0;
    if (!resume) r = reset_scal(ctx);   // a continued run keeps the sticky status
    if (r) return r;
    const int rule = ctx->cfg.batch_rule;
    hipLaunchKernelGGL(batch_init_kernel, dim3(nb), dim3(256), 0, ctx->stream, Upacked, ctx->total,
                       ctx->d_off, ctx->d_n, ctx->d_h, ctx->d_dt, ctx->d_t, ctx->d_steps,
                       ctx->cfg.gamma, cfl, t_end, resume ? 1 : 0, (long long)nsteps_max, rule,
                       rule == PP_DT_RESTART ? ctx->d_bad : nullptr, ctx->d_half);
    HIPCHK(ctx, hipGetLastError());
    ctx->batch_started = true;
    // K steps (3 persistent launches each) captured once in a graph on a
    // private stream, replayed until every problem has retired
    const int K = 8;
    hipStream_t user = ctx->stream, gs = nullptr;
    hipEvent_t ev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // A retired problem (dt = 0) stays retired for the rest of the run.  Once
    // the active set has halved, each class is cut down to its active
    // problems (same kernel shape and LDS as the full class), so the tail of
    // a run launches neither workgroups nor scans for finished lines; every
    // line is still advanced by one workgroup, so the results do not change.
    // The full order is put back before returning.
    const std::vector<int> full_order = ctx->order_host;
    const int full_nclass = ctx->nclass;
    pp_cweno_ctx::LenClass full_cls[3];
    for (int c = 0; c < 3; ++c) full_cls[c] = ctx->cls[c];
    bool compacted = false;
    auto destroy_graph = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    };
    auto cleanup = [&]() -> hipError_t {
        ctx->stream = user;
        destroy_graph();
        hipError_t er = hipSuccess;
        if (compacted) {
            if (gs) er = hipStreamSynchronize(gs);
            ctx->order_host = full_order;
            ctx->nclass = full_nclass;
            for (int c = 0; c < 3; ++c) ctx->cls[c] = full_cls[c];
            if (er == hipSuccess)
                er = hipMemcpy(ctx->d_order, full_order.data(), sizeof(int) * nb, hipMemcpyHostToDevice);
        }
        if (ev) (void)hipEventDestroy(ev);
        if (gs) (void)hipStreamDestroy(gs);
        return er;
    };
    auto capture = [&]() -> int {
        hipError_t ec = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal);
        if (ec != hipSuccess) return hip_fail(ctx, ec, "hipStreamBeginCapture");
        ctx->stream = gs;
        int rc = 0;
        for (int k = 0; k < K && rc == 0; ++k)
            rc = batch_step_launch(ctx, Upacked, ctx->d_dt, true, cfl, t_end, nsteps_max);
        ec = hipStreamEndCapture(gs, &graph);
        ctx->stream = user;
        if (rc) return rc;
        if (ec != hipSuccess) return hip_fail(ctx, ec, "hipStreamEndCapture");
        ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ec != hipSuccess) return hip_fail(ctx, ec, "hipGraphInstantiate");
        return 0;
    };
    // error paths: report the first failure, and a failure of the cleanup
    // after it in the same message
    auto fail_after = [&](int code) -> int {
        const hipError_t ce = cleanup();
        if (ce != hipSuccess) ctx->err += std::string("; cleanup: ") + hipGetErrorString(ce);
        return code;
    };
    hipError_t e = hipStreamCreateWithFlags(&gs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, user);
    if (e == hipSuccess) e = hipStreamWaitEvent(gs, ev, 0);
    if (e != hipSuccess) return fail_after(hip_fail(ctx, e, "graph capture setup"));
    r = capture();
    if (r) return fail_after(r);
    std::vector<double> dts(nb);
    std::vector<int> act;
    act.reserve(nb);
    int compact_ref = nb;
    // a redone step (restart rule) takes a replay slot without advancing, so
    // that rule replays until every problem has retired
    const int64_t max_replays = rule == PP_DT_RESTART ? INT64_MAX : nsteps_max / K + 2;
    for (int64_t rep = 0; rep < max_replays; ++rep) {
        e = hipGraphLaunch(exec, gs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dts.data(), ctx->d_dt, sizeof(double) * nb, hipMemcpyDeviceToHost, gs);
        if (e == hipSuccess) e = hipStreamSynchronize(gs);
        if (e != hipSuccess) return fail_after(hip_fail(ctx, e, "graph replay"));
        int active = 0;
        for (double d : dts) active += d > 0.0;
        if (active == 0) break;
        if (2 * active > compact_ref) continue;
        // cut every class of the full plan down to its active problems
        act.clear();
        int nc = 0;
        for (int c = 0; c < full_nclass; ++c) {
            const int begin = (int)act.size();
            for (int i = full_cls[c].begin; i < full_cls[c].begin + full_cls[c].count; ++i)
                if (dts[full_order[i]] > 0.0) act.push_back(full_order[i]);
            const int count = (int)act.size() - begin;
            if (count == 0) continue;
            ctx->cls[nc].begin = begin;
            ctx->cls[nc].count = count;
            ctx->cls[nc].maxn = full_cls[c].maxn;
            ctx->cls[nc].w = full_cls[c].w;
            ++nc;
        }
        compacted = true;
        ctx->nclass = nc;
        ctx->order_host = act;
        destroy_graph();
        e = hipMemcpyAsync(ctx->d_order, act.data(), sizeof(int) * act.size(), hipMemcpyHostToDevice, gs);
        if (e == hipSuccess) e = hipStreamSynchronize(gs);
        if (e != hipSuccess) return fail_after(hip_fail(ctx, e, "active-set upload"));
        r = capture();
        if (r) return fail_after(r);
        compact_ref = active;
    }
    e = cleanup();
    if (e != hipSuccess) return hip_fail(ctx, e, "restoring the batch order");
    if (steps_out) {
        std::vector<long long> st(nb);
        HIPCHK(ctx, hipMemcpy(st.data(), ctx->d_steps, sizeof(long long) * nb, hipMemcpyDeviceToHost));
        for (int i = 0; i < nb; ++i) steps_out[i] = st[i];
    }
    if (t_out) HIPCHK(ctx, hipMemcpy(t_out, ctx->d_t, sizeof(double) * nb, hipMemcpyDeviceToHost));
    unsigned status = 0;
    HIPCHK(ctx, hipMemcpy(&status, &ctx->scal->status, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (status & 3u) return fail(ctx, PP_ESTATE, "a stage left the admissible set or was not finite");
    return PP_OK;
}

int pp_cweno_batch_run(pp_cweno_ctx* ctx, double* Upacked, double t_end, int64_t nsteps_max,
                       double cfl, int64_t* steps_out) {
    return batch_run_impl(ctx, Upacked, t_end, nsteps_max, cfl, steps_out, nullptr, false);
}

int pp_cweno_batch_continue(pp_cweno_ctx* ctx, double* Upacked, double t_end, int64_t nsteps_max,
                            double cfl, int64_t* steps_out, double* t_out) {
    return batch_run_impl(ctx, Upacked, t_end, nsteps_max, cfl, steps_out, t_out, true);
}

int pp_cweno_status(pp_cweno_ctx* ctx, uint32_t* flags) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    unsigned st = 0;
    HIPCHK(ctx, hipMemcpy(&st, &ctx->scal->status, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (flags) *flags = st;
    if (st) {
        unsigned zero = 0;
        HIPCHK(ctx, hipMemcpy(&ctx->scal->status, &zero, sizeof(unsigned), hipMemcpyHostToDevice));
        if (st & 3u) return fail(ctx, PP_ESTATE, "a stage left the admissible set or was not finite");
    }
    return PP_OK;
}

int pp_cweno_debug_line(pp_cweno_ctx* ctx, const double* U, double* um, double* up, double* flux) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    if (!U) return fail(ctx, PP_EINVAL, "U is NULL");
    if (ctx->cfg.ndim != 1 || ctx->cfg.nbatch > 0) return fail(ctx, PP_EINVAL, "debug_line is 1D only");
    return launch_1d(ctx, U, nullptr, ctx->U2, 0, 0, 0.0, 1.0, nullptr, 0.0, false, um, up, flux);
}

int pp_cweno_tridiag_solve_debug(pp_cweno_ctx* ctx, int64_t n, int cyclic, const double* a,
                                 const double* b, const double* c, const double* r, double* x) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    if (!a || !b || !c || !r || !x) return fail(ctx, PP_EINVAL, "NULL row or solution pointer");
    if (n < 3 || n > 4096) return fail(ctx, PP_EINVAL, "tridiagonal debug solve: 3 <= n <= 4096");
    if (n <= 2048)
        hipLaunchKernelGGL(tridiag_debug_kernel<1>, dim3(1), dim3(64), 0, ctx->stream, a, b, c, r,
                           x, (int)n, cyclic ? 1 : 0);
    else
        hipLaunchKernelGGL(tridiag_debug_kernel<2>, dim3(1), dim3(128), 0, ctx->stream, a, b, c,
                           r, x, (int)n, cyclic ? 1 : 0);
    HIPCHK(ctx, hipGetLastError());
    return PP_OK;
}

int pp_cweno_set_timing(pp_cweno_ctx* ctx, int on) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->timing = on != 0;
    for (int k = 0; k < 3; ++k) ctx->nev[k] = 0;
    return PP_OK;
}

int pp_cweno_get_timing(pp_cweno_ctx* ctx, double* out) {
    if (!ctx) return fail(nullptr, PP_EINVAL, "ctx is NULL");
    if (!out) return fail(ctx, PP_EINVAL, "out is NULL");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < 3; ++k) {
        double tot = 0.0;
        for (int i = 0; i < ctx->nev[k]; ++i) {
            float ms = 0.0f;
            HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->beg[k][i], ctx->ev[k][2 * i + 1]));
            tot += ms;
        }
        out[2 * k] = tot;
        out[2 * k + 1] = ctx->nev[k];
    }
    return PP_OK;
}

const char* pp_cweno_last_error(const pp_cweno_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_init_err.c_str();
}

void pp_cweno_destroy(pp_cweno_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    void* bufs[] = {ctx->U1, ctx->U2, ctx->UA, ctx->UB, ctx->U1B, ctx->U2B, ctx->Lx, ctx->LyB,
                    ctx->Wf, ctx->scal, ctx->d_off, ctx->d_n, ctx->d_h, ctx->d_bc, ctx->d_dt, ctx->d_t,
                    ctx->d_steps,
                    ctx->d_order, ctx->d_counter, ctx->d_dtcopy, ctx->d_tune, ctx->d_bad,
                    ctx->d_half, ctx->chs};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    for (int k = 0; k < 3; ++k)
        for (hipEvent_t e : ctx->ev[k]) (void)hipEventDestroy(e);
    delete ctx;
}

}  // extern "C"
