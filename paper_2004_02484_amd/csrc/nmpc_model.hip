// nmpc_model.hip -- model engine: the double-layer method for further members
// of the paper's PDE class (Sec. 2) on grids of up to kModelMaxNodes nodes:
//
//   heat   w_t = k(w) Lap w + B u with an arbitrary dense B [nodes][m];
//   plate  the thin copper plate of Sec. 5, w_t = alpha Lap w - beta (w - Ta)
//          - rad (w^4 - Ta^4), zero Neumann boundaries by fictitious points
//          (eq. neumann / eq. dis_neumann), the temperatures of the actuator
//          nodes as inputs (those nodes are not states);
//   wave   second order in time, W_tt + damp W_t = k(W) Lap W + B u with the
//          state (W, W_t) of eq. ode; the lower layer's F_x / F_x^T solves
//          eliminate v6 = h v7 - b6 and sweep the reduced system
//          h grad_Wt g - I + h^2 grad_W g (eq. jaco2_sys).
//
// One workgroup owns one instance for the whole solve (persistent): it walks
// the stages with the upper layer of the options -- eq. 1st_jacobi, eq. fgs,
// the backward sweep, or eq. sgs -- solves each stage block by the lower layer
// of Sec. 4.3 (Schur input iteration of Sec. 5.2, point-Jacobi sweeps from
// zero), cuts each pass by the fraction-to-the-boundary rule (eq. alphamax)
// when an input box is set, and takes its convergence decisions itself.
//
// Vectors are kept on the full grid: thread t owns nodes t, t + T, ... (PPT of
// them) in registers; stencil neighbours pass through an LDS copy of the
// vector (two alternating regions, one barrier per stencil). The Laplacian is
// evaluated from the grid geometry: a missing neighbour is zero (Dirichlet)
// or the mirror node (Neumann fictitious point, so a boundary row weights its
// inner neighbour twice, and the transposed operator weights a boundary
// neighbour twice). The plate's actuator nodes hold zero in every state
// vector; its input operator B u = alpha L_su u is the stencil of a vector
// holding u at the actuator nodes, and B^T y is alpha times the transposed
// stencil of y read at the actuator nodes. FP64 throughout.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmpc_model.h"

namespace nmpc {
namespace {

constexpr int kMW = 64;
constexpr int kUpJac = 0, kUpFgs = 1, kUpBgs = 2, kUpSgs = 3;
constexpr int kStOk = 0, kStNoconv = 2, kStNonfinite = 3;

__device__ __forceinline__ unsigned long long mab(double v)
{
    return (unsigned long long)__double_as_longlong(fabs(v));
}
__device__ __forceinline__ double mbd(unsigned long long b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ unsigned long long mmax(unsigned long long x, unsigned long long y)
{
    return x > y ? x : y;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kMW);
    return v;
}
__device__ __forceinline__ unsigned long long wave_umax(unsigned long long v)
{
    for (int o = 32; o >= 1; o >>= 1) v = mmax(v, (unsigned long long)__shfl_xor((long long)v, o, kMW));
    return v;
}

// Neighbour part of (L v)_p (diagonal excluded): the 5-point stencil with
// the boundary rule (Neumann: a missing neighbour is the mirror node).
__device__ __forceinline__ double nsum_at(const double *e, int ix, int iy, const ModelArgs &a)
{
    const int nx = a.nsx, ny = a.nsy;
    double s = 0.0;
    int xe = ix + 1, xw = ix - 1;
    if (a.neumann) {
        if (xe >= nx) xe = ix - 1;
        if (xw < 0) xw = ix + 1;
    }
    if (xe >= 0 && xe < nx) s += a.idx2 * e[iy * nx + xe];
    if (xw >= 0 && xw < nx) s += a.idx2 * e[iy * nx + xw];
    if (ny > 1) {
        int yn = iy + 1, ys = iy - 1;
        if (a.neumann) {
            if (yn >= ny) yn = iy - 1;
            if (ys < 0) ys = iy + 1;
        }
        if (yn >= 0 && yn < ny) s += a.idy2 * e[yn * nx + ix];
        if (ys >= 0 && ys < ny) s += a.idy2 * e[ys * nx + ix];
    }
    return s;
}

// Neighbour part of (L^T v)_p: sum over the neighbours q of L_qp v_q; under
// Neumann boundaries a boundary node q mirrors onto its only inner neighbour,
// so L_qp = 2 / d^2 there.
__device__ __forceinline__ double nsumt_at(const double *e, int ix, int iy, const ModelArgs &a)
{
    const int nx = a.nsx, ny = a.nsy;
    double s = 0.0;
    if (ix + 1 < nx) s += (a.neumann && ix + 1 == nx - 1 ? 2.0 : 1.0) * a.idx2 * e[iy * nx + ix + 1];
    if (ix - 1 >= 0) s += (a.neumann && ix - 1 == 0 ? 2.0 : 1.0) * a.idx2 * e[iy * nx + ix - 1];
    if (ny > 1) {
        if (iy + 1 < ny) s += (a.neumann && iy + 1 == ny - 1 ? 2.0 : 1.0) * a.idy2 * e[(iy + 1) * nx + ix];
        if (iy - 1 >= 0) s += (a.neumann && iy - 1 == 0 ? 2.0 : 1.0) * a.idy2 * e[(iy - 1) * nx + ix];
    }
    return s;
}

template <int PPT>
struct MCtx {
    int tid, T, lane, w, W;
    int p[PPT], ix[PPT], iy[PPT];
    bool node[PPT];   // a grid node
    bool st[PPT];     // a state node (plate: not an actuator node)
    int inp[PPT];     // plate: input index of an actuator node, else -1
    double *ex;       // LDS [2][nodes]
    int flip;
    double *uvec, *ut, *v3, *kun, *red;   // LDS [kModelMaxM] each
    double *redw;                          // LDS [waves][kModelMaxM]
    unsigned long long *nrm;               // LDS [waves][4]
};

// o = neighbour part of L v (TR = false) or of L^T v (TR = true).
template <bool TR, int PPT>
__device__ __forceinline__ void stencil(MCtx<PPT> &c, const ModelArgs &a, const double (&v)[PPT],
                                        double (&o)[PPT])
{
    double *e = c.ex + (size_t)c.flip * a.nodes;
#pragma unroll
    for (int k = 0; k < PPT; ++k)
        if (c.node[k]) e[c.p[k]] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k)
        o[k] = c.node[k] ? (TR ? nsumt_at(e, c.ix[k], c.iy[k], a) : nsum_at(e, c.ix[k], c.iy[k], a))
                         : 0.0;
    c.flip ^= 1;
}

// (B v)_p for a dense B and v in LDS.
template <int PPT>
__device__ __forceinline__ void b_dense(const MCtx<PPT> &c, const ModelArgs &a, const double *v,
                                        double (&o)[PPT])
{
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        double s = 0.0;
        if (c.node[k])
            for (int j = 0; j < a.m; ++j) s += a.B[(size_t)c.p[k] * a.m + j] * v[j];
        o[k] = s;
    }
}

// red[j] = (B^T y)_j for a dense B (block sums; ends with a barrier).
template <int PPT>
__device__ __forceinline__ void bt_dense(MCtx<PPT> &c, const ModelArgs &a, const double (&y)[PPT])
{
    for (int j = 0; j < a.m; ++j) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < PPT; ++k)
            if (c.node[k]) s += a.B[(size_t)c.p[k] * a.m + j] * y[k];
        s = wave_sum(s);
        if (c.lane == 0) c.redw[c.w * kModelMaxM + j] = s;
    }
    __syncthreads();
    if (c.tid < a.m) {
        double s = 0.0;
        for (int ww = 0; ww < c.W; ++ww) s += c.redw[ww * kModelMaxM + c.tid];
        c.red[c.tid] = s;
    }
    __syncthreads();
}

// Stage coefficients of the lower layer (per owned node).
template <int PPT>
struct Coef {
    double invd[PPT];   // 1 / diagonal of the swept matrix (F_x, or eq. jaco2_sys)
    double kc[PPT];     // heat / wave: k(w); plate: unused
    double kl[PPT];     // heat / wave: k' (L w); plate: A_xx diagonal / h
    double lw[PPT];     // heat / wave: lambda (heat) or lambda_V (wave) times k'
};

// Buffers of one stage visit.
struct Visit {
    int b, i, src, dst, xpb, lnb, utb;
    bool res, res_only;
};

template <int MODEL, int PPT>
__device__ void stage_visit(const ModelArgs &a, MCtx<PPT> &c, const Visit &vs,
                            unsigned long long (&acc)[2])
{
    constexpr int NV = MODEL == kModelWave ? 2 : 1;
    const int n = a.nodes, m = a.m, N = a.N, i = vs.i;
    const double h = a.h;
    const size_t so = ((size_t)vs.b * N + i) * a.nxg;
    const size_t uo = ((size_t)vs.b * N + i) * m;
    const bool last = i == N - 1;
    const double *Xc = a.X[vs.src] + so, *Lc = a.LAM[vs.src] + so;
    const double *Xp = i == 0 ? a.x0 + (size_t)vs.b * a.nxg : a.X[vs.xpb] + so - a.nxg;
    const double *Xq = i == 0 ? Xp : a.X[vs.src] + so - a.nxg;
    const double *Ln = last ? nullptr : a.LAM[vs.lnb] + so + a.nxg;
    const double *Lq = last ? nullptr : a.LAM[vs.src] + so + a.nxg;
    const double *xr = a.xref + (size_t)vs.b * n;

    __syncthreads();   // the previous visit's LDS scalars and global writes are done
    double x[PPT][NV], lam[PPT][NV];
#pragma unroll
    for (int k = 0; k < PPT; ++k)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            x[k][v] = c.st[k] ? Xc[c.p[k] + v * n] : 0.0;
            lam[k][v] = c.st[k] ? Lc[c.p[k] + v * n] : 0.0;
        }
    if (c.tid < m) {
        const double u = a.U[vs.src][uo + c.tid];
        c.uvec[c.tid] = u;
        c.ut[c.tid] = vs.utb >= 0 ? a.U[vs.utb][uo + c.tid] : u;
    }
    __syncthreads();

    // ---- KKT rows (Sec. 3.2): b1 = K^x, b2 = K^lambda; red = grad_u f^T lambda
    double b1[PPT][NV], b2[PPT][NV];
    Coef<PPT> K;
    unsigned long long mx = 0, ml = 0;
    auto xprev = [&](int k, int v, bool resv) {
        return (resv ? Xq : Xp)[c.p[k] + v * n];
    };
    auto lnext = [&](int k, int v, bool resv) {
        return last ? 0.0 : (resv ? Lq : Ln)[c.p[k] + v * n];
    };
    if constexpr (MODEL == kModelPlate) {
        double w[PPT], Lw[PPT], lt[PPT], LTl[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            w[k] = c.st[k] ? x[k][0] : (c.inp[k] >= 0 ? c.uvec[c.inp[k]] : 0.0);
            lt[k] = lam[k][0];   // zero at the actuator nodes
        }
        stencil<false>(c, a, w, Lw);
        stencil<true>(c, a, lt, LTl);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (c.inp[k] >= 0) c.red[c.inp[k]] = a.alpha * LTl[k];   // (B^T lambda)_j
            const double xv = x[k][0], lv = lam[k][0];
            double kx = 0.0, kl = 0.0, kxr = 0.0, klr = 0.0;
            if (c.st[k]) {
                const double f = a.alpha * (Lw[k] + a.lpp * xv) - a.beta * (xv - a.tamb) -
                                 a.rad * (xv * xv * xv * xv - a.tamb * a.tamb * a.tamb * a.tamb);
                kx = xprev(k, 0, false) - xv + h * f;
                kxr = xprev(k, 0, true) - xv + h * f;
                const double rest = h * (a.q * (xv - xr[c.p[k]]) + a.alpha * (LTl[k] + a.lpp * lv) -
                                         (a.beta + 4.0 * a.rad * xv * xv * xv) * lv);
                kl = lnext(k, 0, false) - lv + rest;
                klr = lnext(k, 0, true) - lv + rest;
            }
            b1[k][0] = kx;
            b2[k][0] = kl;
            mx = mmax(mx, mab(kxr));
            ml = mmax(ml, mab(klr));
            // lower-layer coefficients: F_x diagonal, A_xx / h
            const double d = -1.0 + h * (a.alpha * a.lpp - a.beta - 4.0 * a.rad * xv * xv * xv);
            K.invd[k] = c.st[k] ? 1.0 / d : 0.0;
            K.kl[k] = a.q - 12.0 * a.rad * xv * xv * lv;
            K.kc[k] = 0.0;
            K.lw[k] = 0.0;
        }
        __syncthreads();   // red written by the actuator nodes' owners
    } else if constexpr (MODEL == kModelHeat) {
        double xv[PPT], Lx[PPT], g[PPT], LTg[PPT], Bu[PPT];
        const double kp = a.k0 * a.k1;
#pragma unroll
        for (int k = 0; k < PPT; ++k) xv[k] = x[k][0];
        stencil<false>(c, a, xv, Lx);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            Lx[k] += a.lpp * xv[k];
            K.kc[k] = a.k0 * (1.0 + a.k1 * xv[k]);
            g[k] = K.kc[k] * lam[k][0];
        }
        stencil<true>(c, a, g, LTg);
        b_dense(c, a, c.uvec, Bu);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            double kx = 0.0, kl = 0.0, kxr = 0.0, klr = 0.0;
            if (c.st[k]) {
                const double f = K.kc[k] * Lx[k] + Bu[k];
                kx = xprev(k, 0, false) - xv[k] + h * f;
                kxr = xprev(k, 0, true) - xv[k] + h * f;
                const double rest = h * (a.q * (xv[k] - xr[c.p[k]]) + LTg[k] + a.lpp * g[k] +
                                         kp * Lx[k] * lam[k][0]);
                kl = lnext(k, 0, false) - lam[k][0] + rest;
                klr = lnext(k, 0, true) - lam[k][0] + rest;
            }
            b1[k][0] = kx;
            b2[k][0] = kl;
            mx = mmax(mx, mab(kxr));
            ml = mmax(ml, mab(klr));
            const double d = -1.0 + h * (K.kc[k] * a.lpp + kp * Lx[k]);
            K.invd[k] = c.st[k] ? 1.0 / d : 0.0;
            K.kl[k] = kp * Lx[k];
            K.lw[k] = kp * lam[k][0];
        }
        double lv[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) lv[k] = lam[k][0];
        bt_dense(c, a, lv);
    } else {   // wave
        double W[PPT], LW[PPT], g[PPT], LTg[PPT], Bu[PPT];
        const double kp = a.k0 * a.k1;
#pragma unroll
        for (int k = 0; k < PPT; ++k) W[k] = x[k][0];
        stencil<false>(c, a, W, LW);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            LW[k] += a.lpp * W[k];
            K.kc[k] = a.k0 * (1.0 + a.k1 * W[k]);
            g[k] = K.kc[k] * lam[k][1];
        }
        stencil<true>(c, a, g, LTg);
        b_dense(c, a, c.uvec, Bu);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            double kx0 = 0.0, kx1 = 0.0, kl0 = 0.0, kl1 = 0.0;
            unsigned long long mxk = 0, mlk = 0;
            if (c.st[k]) {
                const double V = x[k][1], lW = lam[k][0], lV = lam[k][1];
                const double gg = K.kc[k] * LW[k] - a.damp * V + Bu[k];
                kx0 = xprev(k, 0, false) - W[k] + h * V;
                kx1 = xprev(k, 1, false) - V + h * gg;
                const double r0 = h * (a.q * (W[k] - xr[c.p[k]]) + LTg[k] + a.lpp * g[k] +
                                       kp * LW[k] * lV);
                const double r1 = h * (a.qv * V + lW - a.damp * lV);
                kl0 = lnext(k, 0, false) - lW + r0;
                kl1 = lnext(k, 1, false) - lV + r1;
                mxk = mmax(mab(xprev(k, 0, true) - W[k] + h * V),
                           mab(xprev(k, 1, true) - V + h * gg));
                mlk = mmax(mab(lnext(k, 0, true) - lW + r0), mab(lnext(k, 1, true) - lV + r1));
            }
            b1[k][0] = kx0;
            b1[k][NV - 1] = kx1;
            b2[k][0] = kl0;
            b2[k][NV - 1] = kl1;
            mx = mmax(mx, mxk);
            ml = mmax(ml, mlk);
            // reduced system diagonal: -(1 + h damp) + h^2 (k L_pp + k' L W)
            const double d = -(1.0 + h * a.damp) + h * h * (K.kc[k] * a.lpp + kp * LW[k]);
            K.invd[k] = c.st[k] ? 1.0 / d : 0.0;
            K.kl[k] = kp * LW[k];
            K.lw[k] = kp * lam[k][1];
        }
        double lv[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) lv[k] = lam[k][1];
        bt_dense(c, a, lv);
    }

    // ---- input rows and norms
    unsigned long long mu = 0;
    if (c.tid < m) {
        const double u = c.uvec[c.tid];
        double bg = 0.0;
        if (a.tau > 0.0) bg = -a.tau / (u - a.ulo) + a.tau / (a.uhi - u);
        double ur = 0.0;
        if (MODEL == kModelPlate) ur = xr[a.act[c.tid]];
        const double ku = h * (a.r * (u - ur) + c.red[c.tid] + bg);
        c.kun[c.tid] = ku + a.gamma * (u - c.ut[c.tid]);
        c.v3[c.tid] = 0.0;
        mu = mab(ku);
    }
    if (vs.res) {
        mx = wave_umax(mx);
        ml = wave_umax(ml);
        mu = wave_umax(mu);
        if (c.lane == 0) {
            c.nrm[c.w * 4 + 0] = mx;
            c.nrm[c.w * 4 + 1] = ml;
            c.nrm[c.w * 4 + 2] = mu;
        }
    }
    __syncthreads();
    if (vs.res && c.tid == 0) {
        unsigned long long ax = 0, al = 0, au = 0;
        for (int ww = 0; ww < c.W; ++ww) {
            ax = mmax(ax, c.nrm[ww * 4 + 0]);
            al = mmax(al, c.nrm[ww * 4 + 1]);
            au = mmax(au, c.nrm[ww * 4 + 2]);
        }
        const double dx_ = mbd(ax), dl_ = mbd(al), du_ = mbd(au);
        double rp = fmax(fmax(dx_, du_), dl_);
        double rs = fmax(fmax(dx_, du_ / (h * a.r)), dl_ / h);
        if (ax >= 0x7FF0000000000000ull || al >= 0x7FF0000000000000ull ||
            au >= 0x7FF0000000000000ull)
            rs = rp = __longlong_as_double(0x7FF8000000000000ll);
        acc[0] = mmax(acc[0], mab(rs));
        acc[1] = mmax(acc[1], mab(rp));
    }
    if (vs.res_only) return;

    // ---- lower layer (Sec. 4.3): F_x / F_x^T solves by n_sw point-Jacobi sweeps from 0
    // y = F_x^{-1} r (approximately), r and y with NV entries per node
    auto solve_f = [&](const double (&r)[PPT][NV], double (&y)[PPT][NV]) {
        if constexpr (MODEL == kModelWave) {
            // v6 = h v7 - b6; (-(1 + h damp) I + h^2 G) v7 = b7 + h G b6, G = diag(k) L + diag(k' L W)
            double b6[PPT], nb[PPT], rhs[PPT], v7[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) b6[k] = r[k][0];
            stencil<false>(c, a, b6, nb);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const double Gb6 = K.kc[k] * (nb[k] + a.lpp * b6[k]) + K.kl[k] * b6[k];
                rhs[k] = c.st[k] ? r[k][1] + h * Gb6 : 0.0;
                v7[k] = rhs[k] * K.invd[k];
            }
            for (int s = 1; s < a.n_sw; ++s) {
                stencil<false>(c, a, v7, nb);
#pragma unroll
                for (int k = 0; k < PPT; ++k) v7[k] = (rhs[k] - h * h * K.kc[k] * nb[k]) * K.invd[k];
            }
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                y[k][NV - 1] = v7[k];
                y[k][0] = c.st[k] ? h * v7[k] - b6[k] : 0.0;
            }
        } else {
            double yy[PPT], nb[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) yy[k] = r[k][0] * K.invd[k];
            for (int s = 1; s < a.n_sw; ++s) {
                stencil<false>(c, a, yy, nb);
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const double off = MODEL == kModelPlate ? h * a.alpha * nb[k] : h * K.kc[k] * nb[k];
                    yy[k] = (r[k][0] - off) * K.invd[k];
                }
            }
#pragma unroll
            for (int k = 0; k < PPT; ++k) y[k][0] = yy[k];
        }
    };
    auto solve_ft = [&](const double (&r)[PPT][NV], double (&y)[PPT][NV]) {
        if constexpr (MODEL == kModelWave) {
            // v6 = h G^T v7 - b6; (-(1 + h damp) I + h^2 G^T) v7 = b7 + h b6
            double rhs[PPT], v7[PPT], z[PPT], nb[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                rhs[k] = c.st[k] ? r[k][1] + h * r[k][0] : 0.0;
                v7[k] = rhs[k] * K.invd[k];
            }
            for (int s = 1; s < a.n_sw; ++s) {
#pragma unroll
                for (int k = 0; k < PPT; ++k) z[k] = K.kc[k] * v7[k];
                stencil<true>(c, a, z, nb);
#pragma unroll
                for (int k = 0; k < PPT; ++k) v7[k] = (rhs[k] - h * h * nb[k]) * K.invd[k];
            }
#pragma unroll
            for (int k = 0; k < PPT; ++k) z[k] = K.kc[k] * v7[k];
            stencil<true>(c, a, z, nb);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const double Gt = nb[k] + a.lpp * z[k] + K.kl[k] * v7[k];   // (G^T v7)_p
                y[k][NV - 1] = v7[k];
                y[k][0] = c.st[k] ? h * Gt - r[k][0] : 0.0;
            }
        } else {
            double yy[PPT], z[PPT], nb[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) yy[k] = r[k][0] * K.invd[k];
            for (int s = 1; s < a.n_sw; ++s) {
#pragma unroll
                for (int k = 0; k < PPT; ++k) z[k] = MODEL == kModelPlate ? yy[k] : K.kc[k] * yy[k];
                stencil<true>(c, a, z, nb);
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const double off = MODEL == kModelPlate ? h * a.alpha * nb[k] : h * nb[k];
                    yy[k] = (r[k][0] - off) * K.invd[k];
                }
            }
#pragma unroll
            for (int k = 0; k < PPT; ++k) y[k][0] = yy[k];
        }
    };
    // o = A_xx y = h grad_xx^2 H y
    auto axx = [&](const double (&y)[PPT][NV], double (&o)[PPT][NV]) {
        if constexpr (MODEL == kModelPlate) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) o[k][0] = h * K.kl[k] * y[k][0];
        } else {
            // first block: h (q y + k' (lam . L y + L^T (lam . y)))
            double y0[PPT], z[PPT], n1[PPT], n2[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                y0[k] = y[k][0];
                z[k] = K.lw[k] * y0[k];
            }
            stencil<false>(c, a, y0, n1);
            stencil<true>(c, a, z, n2);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const double Ly = n1[k] + a.lpp * y0[k];
                const double LTz = n2[k] + a.lpp * z[k];
                o[k][0] = c.st[k] ? h * (a.q * y0[k] + K.lw[k] * Ly + LTz) : 0.0;
                if constexpr (NV == 2) o[k][NV - 1] = h * a.qv * y[k][NV - 1];
            }
        }
    };
    // o = F_u v (v in LDS)
    auto fu_apply = [&](const double *v, double (&o)[PPT][NV]) {
        if constexpr (MODEL == kModelPlate) {
            double w[PPT], nb[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) w[k] = c.inp[k] >= 0 ? v[c.inp[k]] : 0.0;
            stencil<false>(c, a, w, nb);
#pragma unroll
            for (int k = 0; k < PPT; ++k) o[k][0] = c.st[k] ? h * a.alpha * nb[k] : 0.0;
        } else {
            double Bv[PPT];
            b_dense(c, a, v, Bv);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if constexpr (NV == 2) o[k][0] = 0.0;
                o[k][NV - 1] = c.st[k] ? h * Bv[k] : 0.0;
            }
        }
    };
    // red[j] = (F_u^T y)_j / h (ends with a barrier)
    auto fut_apply = [&](const double (&y)[PPT][NV]) {
        if constexpr (MODEL == kModelPlate) {
            double yy[PPT], nb[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) yy[k] = y[k][0];
            stencil<true>(c, a, yy, nb);
#pragma unroll
            for (int k = 0; k < PPT; ++k)
                if (c.inp[k] >= 0) c.red[c.inp[k]] = a.alpha * nb[k];
            __syncthreads();
        } else {
            double yy[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) yy[k] = y[k][NV - 1];
            bt_dense(c, a, yy);
        }
    };

    double auu = 0.0;
    if (c.tid < m) {
        const double u = c.uvec[c.tid];
        double hb = 0.0;
        if (a.tau > 0.0) {
            const double lo = u - a.ulo, hi = a.uhi - u;
            hb = a.tau / (lo * lo) + a.tau / (hi * hi);
        }
        auu = h * (a.r + hb) + a.gamma;
    }
    double y5[PPT][NV], y4[PPT][NV], cc[PPT][NV], t[PPT][NV];
    for (int s = 0; s < a.n_schur; ++s) {
        fu_apply(c.v3, t);
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int v = 0; v < NV; ++v) cc[k][v] = t[k][v] - b1[k][v];
        solve_f(cc, y5);
        axx(y5, t);
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int v = 0; v < NV; ++v) cc[k][v] = -b2[k][v] - t[k][v];
        solve_ft(cc, y4);
        fut_apply(y4);
        if (c.tid < m) c.v3[c.tid] = (c.kun[c.tid] + h * c.red[c.tid]) / auu;
        __syncthreads();
    }
    fu_apply(c.v3, t);
#pragma unroll
    for (int k = 0; k < PPT; ++k)
#pragma unroll
        for (int v = 0; v < NV; ++v) cc[k][v] = b1[k][v] - t[k][v];
    solve_f(cc, y5);   // dx
    axx(y5, t);
#pragma unroll
    for (int k = 0; k < PPT; ++k)
#pragma unroll
        for (int v = 0; v < NV; ++v) cc[k][v] = b2[k][v] - t[k][v];
    solve_ft(cc, y4);  // dlambda

    // ---- update S_new = S - ds (alpha = 1; the pass is cut afterwards)
    double *Xn = a.X[vs.dst] + so, *Lw = a.LAM[vs.dst] + so;
#pragma unroll
    for (int k = 0; k < PPT; ++k)
        if (c.st[k]) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                Xn[c.p[k] + v * n] = x[k][v] - y5[k][v];
                Lw[c.p[k] + v * n] = lam[k][v] - y4[k][v];
            }
        }
    if (c.tid < m) {
        const double u = c.uvec[c.tid], d = c.v3[c.tid];
        a.U[vs.dst][uo + c.tid] = u - d;
        double l = 1.0;   // fraction-to-the-boundary limit (eq. alphamax) of this input
        if (a.tau > 0.0) {
            if (d > 0.0) l = 0.995 * (u - a.ulo) / d;
            else if (d < 0.0) l = 0.995 * (a.uhi - u) / (-d);
            l = fmax(l, 0.0);
        }
        c.red[c.tid] = l;
    }
    __syncthreads();
    if (c.tid == 0 && a.tau > 0.0) {
        double l = 1.0;
        for (int j = 0; j < m; ++j) l = fmin(l, c.red[j]);
        a.lim[(size_t)vs.b * N + i] = l;
    }
}

// S_to = S_from + alpha (S_to - S_from) over the whole instance (alpha < 1).
template <int PPT>
__device__ void blend(const ModelArgs &a, const MCtx<PPT> &c, int b, int from, int to, double alpha)
{
    const size_t nx = (size_t)a.N * a.nxg, nu = (size_t)a.N * a.m;
    const size_t xo = (size_t)b * nx, uo = (size_t)b * nu;
    for (size_t t = c.tid; t < nx; t += c.T) {
        const double xf = a.X[from][xo + t], lf = a.LAM[from][xo + t];
        a.X[to][xo + t] = xf + alpha * (a.X[to][xo + t] - xf);
        a.LAM[to][xo + t] = lf + alpha * (a.LAM[to][xo + t] - lf);
    }
    for (size_t t = c.tid; t < nu; t += c.T) {
        const double uf = a.U[from][uo + t];
        a.U[to][uo + t] = uf + alpha * (a.U[to][uo + t] - uf);
    }
}

template <int PPT>
__device__ double pass_alpha(const ModelArgs &a, MCtx<PPT> &c, int b)
{
    __syncthreads();   // every stage's limit is written
    double l = 1.0;
    for (int i = c.tid; i < a.N; i += c.T) l = fmin(l, a.lim[(size_t)b * a.N + i]);
    // block minimum of values in (0, 1]: max of the bit patterns of 2 - l
    unsigned long long v = wave_umax(mab(2.0 - l));
    if (c.lane == 0) c.nrm[c.w * 4 + 3] = v;
    __syncthreads();
    unsigned long long mxv = 0;
    for (int ww = 0; ww < c.W; ++ww) mxv = mmax(mxv, c.nrm[ww * 4 + 3]);
    __syncthreads();
    return 2.0 - mbd(mxv);
}

// One pass of the upper layer over the stages: dir 0 (Jacobi: all stages from
// src), +1 forward or -1 backward Gauss-Seidel (x_{i-1} of a forward pass and
// lambda_{i+1} of a backward pass come from the stages already visited).
template <int MODEL, int PPT>
__device__ void run_pass(const ModelArgs &a, MCtx<PPT> &c, int b, int dir, int src, int dst,
                         int utb, bool res, bool res_only, unsigned long long (&acc)[2])
{
    Visit vs;
    vs.b = b;
    vs.src = src;
    vs.dst = dst;
    vs.xpb = dir > 0 ? dst : src;
    vs.lnb = dir < 0 ? dst : src;
    vs.utb = utb;
    vs.res = res;
    vs.res_only = res_only;
    for (int t = 0; t < a.N; ++t) {
        vs.i = dir >= 0 ? t : a.N - 1 - t;
        stage_visit<MODEL, PPT>(a, c, vs, acc);
    }
}

template <int MODEL, int PPT>
__global__ void __launch_bounds__(PPT == 1 ? 1024 : 512) k_model(const ModelArgs a)
{
    extern __shared__ __align__(16) double mlds[];
    const int b = blockIdx.x;
    if (b >= a.count) return;
    MCtx<PPT> c;
    c.tid = threadIdx.x;
    c.T = blockDim.x;
    c.lane = c.tid & (kMW - 1);
    c.w = c.tid / kMW;
    c.W = c.T / kMW;
    c.ex = mlds;
    c.uvec = mlds + 2 * a.nodes;
    c.ut = c.uvec + kModelMaxM;
    c.v3 = c.ut + kModelMaxM;
    c.kun = c.v3 + kModelMaxM;
    c.red = c.kun + kModelMaxM;
    c.redw = c.red + kModelMaxM;
    c.nrm = reinterpret_cast<unsigned long long *>(c.redw + (size_t)c.W * kModelMaxM);
    c.flip = 0;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int p = c.tid + k * c.T;
        c.p[k] = p;
        c.node[k] = p < a.nodes;
        c.ix[k] = p % a.nsx;
        c.iy[k] = p / a.nsx;
        c.inp[k] = (MODEL == kModelPlate && c.node[k]) ? a.nodeinp[p] : -1;
        c.st[k] = c.node[k] && c.inp[k] < 0;
    }
    int *info = a.info_i + (size_t)b * 4;
    unsigned long long acc[2] = {0, 0};
    unsigned long long *bc = c.nrm + 2;   // broadcast slots (words 2, 3 of wave 0's norms)
    auto reduce_acc = [&](double &rs, double &rp) {
        __syncthreads();
        if (c.tid == 0) { c.nrm[0] = acc[0]; c.nrm[1] = acc[1]; }
        __syncthreads();
        rs = mbd(c.nrm[0]);
        rp = mbd(c.nrm[1]);
        __syncthreads();
    };
    (void)bc;
    if (a.residual_only) {
        run_pass<MODEL, PPT>(a, c, b, 0, 0, 1, -1, true, true, acc);
        double rs, rp;
        reduce_acc(rs, rp);
        if (c.tid == 0) {
            a.info_d[2 * b] = rs;
            a.info_d[2 * b + 1] = rp;
        }
        return;
    }
    const int up = a.upper;
    const int d1 = up == kUpJac ? 0 : (up == kUpFgs ? 1 : -1);
    int cur = 0, j = 0, status = -1, evals = 0;
    double rs = 0.0, rp = 0.0;
    for (;;) {
        const int oth = cur ^ 1;
        acc[0] = acc[1] = 0;
        run_pass<MODEL, PPT>(a, c, b, d1, cur, oth, -1, true, false, acc);
        ++evals;
        reduce_acc(rs, rp);
        const double r = a.res_paper ? rp : rs;
        if (!(r <= 1.7976931348623157e308)) { status = kStNonfinite; break; }
        if (r <= a.tol) { status = kStOk; break; }
        if (j >= a.max_iter) { status = kStNoconv; break; }
        if (a.tau > 0.0) {
            const double al = pass_alpha(a, c, b);
            if (al < 1.0) blend(a, c, b, cur, oth, al);
        }
        if (up == kUpSgs) {
            // forward pass from the backward pass's result into buffer cur; the
            // regularization reference u~ = u^j is read from cur before each
            // stage overwrites it
            __syncthreads();
            run_pass<MODEL, PPT>(a, c, b, 1, oth, cur, cur, false, false, acc);
            ++evals;
            if (a.tau > 0.0) {
                const double al = pass_alpha(a, c, b);
                if (al < 1.0) blend(a, c, b, oth, cur, al);
            }
        } else {
            cur = oth;
        }
        ++j;
        __syncthreads();
    }
    __syncthreads();
    if (c.tid == 0) {
        info[0] = j;
        info[1] = status;
        info[2] = cur;
        info[3] = evals;
        a.info_d[2 * b] = rs;
        a.info_d[2 * b + 1] = rp;
    }
    // the returned iterate S^j (buffer cur) to the dense outputs; the plate's
    // actuator nodes take the inputs' values (the node temperatures)
    if (a.out_x) {
        const size_t nxs = (size_t)a.N * a.nxg, nus = (size_t)a.N * a.m;
        for (size_t t = c.tid; t < nxs; t += c.T) {
            double v = a.X[cur][(size_t)b * nxs + t];
            double l = a.LAM[cur][(size_t)b * nxs + t];
            if (MODEL == kModelPlate) {
                const int p = (int)(t % a.nxg), ii = (int)(t / a.nxg);
                const int jin = a.nodeinp[p];
                if (jin >= 0) {
                    v = a.U[cur][((size_t)b * a.N + ii) * a.m + jin];
                    l = 0.0;
                }
            }
            a.out_x[(size_t)b * nxs + t] = v;
            a.out_lam[(size_t)b * nxs + t] = l;
        }
        for (size_t t = c.tid; t < nus; t += c.T) a.out_u[(size_t)b * nus + t] = a.U[cur][(size_t)b * nus + t];
    }
}

__global__ void k_model_init(const ModelArgs a, const ModelInit w)
{
    const size_t nx = (size_t)a.count * a.N * a.nxg, nu = (size_t)a.count * a.N * a.m;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < nx; t += stride) {
        const size_t p = t % a.nxg, b = t / ((size_t)a.N * a.nxg);
        const bool state = a.model != kModelPlate || a.nodeinp[p] < 0;
        a.X[0][t] = state ? (w.wx ? w.wx[t] : a.x0[b * a.nxg + p]) : 0.0;
        a.LAM[0][t] = state && w.wl ? w.wl[t] : 0.0;
        if (!state) {   // never written by the passes: zero in both buffers
            a.X[1][t] = 0.0;
            a.LAM[1][t] = 0.0;
        }
    }
    const double marg = 0.005 * (a.uhi - a.ulo);
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < nu; t += stride) {
        double u = w.wu ? w.wu[t] : w.u_cold;
        if (w.project) {   // strictly feasible S^0 (Sec. 4.2)
            if (u < a.ulo + marg) u = a.ulo + marg;
            if (u > a.uhi - marg) u = a.uhi - marg;
        }
        a.U[0][t] = u;
    }
}

}  // namespace

const void *model_init_kernel() { return (const void *)&k_model_init; }

const void *model_kernel(int model, int ppt)
{
#define NMPC_MK(MD)                                                                 \
    if (model == MD) {                                                              \
        if (ppt == 1) return (const void *)&k_model<MD, 1>;                         \
        if (ppt == 4) return (const void *)&k_model<MD, 4>;                         \
        if (ppt == 8) return (const void *)&k_model<MD, 8>;                         \
    }
    NMPC_MK(kModelHeat)
    NMPC_MK(kModelPlate)
    NMPC_MK(kModelWave)
#undef NMPC_MK
    return nullptr;
}

}  // namespace nmpc
