// nmpc_kernels.hip -- gfx950 kernels of the double-layer Jacobi NMPC solver
// for a batch of instances of one problem.
//
// One workgroup owns one (instance, stage) unit of one upper iteration
// (eq. 1st_jacobi: every stage block is solved from S^k alone, so all units of
// an iteration are independent). Per unit and upper iteration the kernel fuses
// (device code in nmpc_stage.h):
//   1. the KKT rows K_i (Sec. 3.2) in FP64 and their inf-norms, stored per
//      stage and max-reduced per instance by the next launch's decision;
//   2. the lower layer (Sec. 4.3): stage coefficients, n_schur Schur input
//      iterations with diagonal A_uu (Sec. 5.2), each F_x / F_x^T solve by
//      n_sweep point-Jacobi sweeps from zero (Lemma lemma_jaco), then the
//      saddle solve of eq. step2 / eq. coff;
//   3. the update S^{k+1} = S^k - ds (alpha = 1), written to the other buffer.
// The lower layer runs in T (float in the FP32-sweep kernel, double in the
// FP64 kernel); S, K, the norms and the convergence test are always FP64.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "nmpc_device.h"
#include "nmpc_stage.h"

namespace nmpc {

template <int PREC, int CX, int RY, int WB, int OCC, int LX, int LY>
__global__ void __launch_bounds__(kWave * WB, OCC) k_iterate(const IterArgs a)
{
    using T = typename std::conditional<PREC == kModeFp32, float, double>::type;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Ctx c;
    c.lds = lds_raw;
    tile_setup<T, CX, RY, LX, LY>(c, a.P);

    const int k = a.residual_only ? 0 : *(volatile const int *)(a.ctr) + a.kofs;
    // XCD-aware unit order: consecutive workgroup ids go to different XCDs, so
    // give each XCD a contiguous run of units (neighbouring stages of one
    // instance then share that XCD's L2 for the x_{i-1} / lambda_{i+1} reads).
    const int bid = blockIdx.x;
    const int unit = (bid & 7) * a.per_xcd + (bid >> 3);
    if (unit < a.units) {
        const int N = a.P.N, n = a.P.n, M = LX * LY;
        const int b = a.res_first_stage ? unit : unit / N, i = a.res_first_stage ? 0 : unit % N;
        Decision d;
        if (a.residual_only) {
            d.work = true; d.j = 0; d.slot = a.res_slot; d.eval_only = false; d.redo = false;
        } else {
            d = decide<PREC>(a, c, b, i, k, N, (long long)b * N);
        }
        if (d.work) {
            StageLoc v = jacobi_loc(d.j & 1);
            v.tgx = a.gx;   // tables loaded after the stage's loads are issued
            v.tgy = a.gy;
            v.defer_norms = true;
            v.xp_lds = a.xp_lds != 0;
            v.so = (long long)b * N * n;
            v.uo = (long long)b * N * M;
            v.xo = (long long)b * n;
            v.xro = (long long)b * a.xref_inst_stride + (long long)i * a.xref_stage_stride;
            v.res_at = (long long)d.slot * a.rslot + (long long)b * N + i;
            v.res_only = d.eval_only;
            if (d.redo && a.du) v.du_at = b;
            if (a.P.tau > 0.0 && !a.residual_only && !d.eval_only) {
                v.box_at = (long long)b * N + i;
                if (i == 0 && c.tid == 0) a.aupd[b] = k + 1;   // this launch updates b
            }
            v.i = i;
            v.last = i == N - 1;
            unsigned long long acc[2] = {0, 0};
            stage_body<T, CX, RY, LX, LY, CX == 4>(a, a.P, v, c, acc);
        }
    }
}

// Input box: after an iteration launch, the fraction-to-the-boundary rule
// (eq. eq_alphamax) with alpha global over an instance's stages. The launch
// wrote the alpha = 1 step S^{j+1} = S^j - ds and each stage's limit; where
// their minimum alpha is below 1 the step is scaled in place,
// S^{j+1} = S^j + alpha (S^{j+1} - S^j). One workgroup per (instance, stage),
// in the iteration kernel's unit order; instances that did not update in this
// launch, or whose alpha is 1, return at once.
__global__ void __launch_bounds__(256) k_box_apply(const IterArgs a)
{
    __shared__ double red[256];
    const int k = *(volatile const int *)(a.ctr) + a.kofs;
    const int bid = blockIdx.x;
    const int unit = (bid & 7) * a.per_xcd + (bid >> 3);
    if (unit >= a.units) return;
    const int N = a.P.N, n = a.P.n, M = a.P.m;
    const int b = unit / N, i = unit % N;
    if (a.aupd[b] != k + 1) return;
    double l = 1.0;
    for (int t = threadIdx.x; t < N; t += blockDim.x) l = fmin(l, a.apart[(size_t)b * N + t]);
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const double alpha = red[0];
    if (!(alpha < 1.0)) return;
    const int src = a.st[((k + 1) & 1) * a.B + b].j & 1, dst = src ^ 1;
    const size_t so = ((size_t)b * N + i) * n, uo = ((size_t)b * N + i) * M;
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
        const double xs = a.X[src][so + p], ls = a.LAM[src][so + p];
        a.X[dst][so + p] = xs + alpha * (a.X[dst][so + p] - xs);
        a.LAM[dst][so + p] = ls + alpha * (a.LAM[dst][so + p] - ls);
    }
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const double us = a.U[src][uo + j];
        a.U[dst][uo + j] = us + alpha * (a.U[dst][uo + j] - us);
    }
}

// Block-wide maximum of a non-negative double, returned to every thread,
// through word 3 of each wave's norm slots; successive calls must be
// separated by a barrier.
__device__ __forceinline__ double block_max_nonneg(double v, Ctx &c, unsigned long long *nrm)
{
    const unsigned long long m = wave_max64(abits(v), c.lane);
    if (c.lane == 0) nrm[c.w * 4 + 3] = m;
    __syncthreads();
    unsigned long long a = 0;
    for (int ww = 0; ww < c.W; ++ww) a = umax64(a, nrm[ww * 4 + 3]);
    return bits2d(a);
}

// Chebyshev weights of the semi-iterative method (Golub & Varga) for a
// fixed-point sweep x <- G x + g whose G has a real spectrum in [-mu, mu]:
// x^1 = G x^0 + g, x^{s+1} = x^{s-1} + w_{s+1} (G x^s + g - x^{s-1}) with
// w_2 = 1 / (1 - mu^2 / 2) and w_{s+1} = 1 / (1 - mu^2 w_s / 4).
__device__ __forceinline__ double cheb_next(int s, double w, double mu2)
{
    return s == 0 ? 1.0 / (1.0 - 0.5 * mu2) : 1.0 / (1.0 - 0.25 * mu2 * w);
}

// Consistent start from an input trajectory u (already in buffer 0): the
// states follow the backward-Euler model of eq. nlp, x_i = x_{i-1} + h f(u_i,
// x_i), solved stage by stage (K^x_i = 0), and the costates follow the
// adjoint recursion K^lam_i = 0 of Sec. 3.2 solved from i = N down to 1, i.e.
// F_x^T lam_i = -(lam_{i+1} + h q (x_i - xref_i)). Both solves are point-Jacobi
// sweeps in FP64 (for the state: on the implicit equation with k(x) taken at
// the current sweep), accelerated by Chebyshev weights. With k frozen, both
// sweep matrices are diagonal scalings of the symmetric stencil (similar to
// symmetric matrices, so their spectra are real) and their row sums bound the
// spectral radius: h k c0 / (1 + h k c0) for the state, c0 h k / |d| for the
// costate (d: the diagonal of F_x), about 0.44 at the stage length used here,
// which the weights bring to about 0.23 per sweep. The bound is taken per
// stage from the sweep's starting point, with 2 % margin; a spectrum slightly
// wider than the bound still converges, only more slowly. The costate sweeps
// start from the lambda already in buffer 0 (a supplied guess, or 0). a.n_sw
// sweeps per stage for the states, a.n_sw_lam for the costates. One
// workgroup per instance.
// The start's KKT residual comes out of the same pass: after each stage's
// sweeps the kernel evaluates that stage's rows (K^x from the built state,
// K^lam and K^u from the built costate) and writes the stage norms into
// residual slot 0, as the residual kernel would.
template <int CX, int RY, int WB, int LX, int LY>
__global__ void __launch_bounds__(kWave * WB) k_rollout(const IterArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Ctx c;
    c.lds = lds_raw;
    c.tid = threadIdx.x;
    c.lane = c.tid & (kWave - 1);
    c.cl = c.lane & 15;
    c.w = c.tid / kWave;
    c.W = blockDim.x / kWave;
    c.G = c.w * 4 + (c.lane >> 4);
    c.GT = c.W * 4;
    c.Gv = (a.P.nsy + RY - 1) / RY;
    c.flip = 0;
    c.ax = a.P.idx2;
    c.ay = a.P.idy2;
    c.off = lds_layout(c.GT, c.W, CX, 8, LX, LY, RY);
    const DevProblem &P = a.P;
    constexpr int M = LX * LY;
    const int b = blockIdx.x;
    if (b >= a.units) return;
    double *uvec = lds_ptr<double>(c, c.off.uvec);
    load_tables<CX, RY, LX, LY>(c, a.gx, a.gy, P.nsx, P.nsy);
    const int n = P.n, sx = 16 * CX;
    const int ix0 = c.cl * CX, iy0 = c.G * RY;
    auto valid = [&](int t, int q) { return ix0 + q < P.nsx && iy0 + t < P.nsy; };
    auto pidx = [&](int t, int q) { return (iy0 + t) * sx + ix0 + q; };
    const double h = P.h, kp = P.k0 * P.k1;
    const int nsw = a.n_sw, nswl = a.n_sw_lam > 0 ? a.n_sw_lam : a.n_sw;
    unsigned long long *nrm = lds_ptr<unsigned long long>(c, c.off.nrm);

    // ---- states, forward in the horizon
    // Each stage starts with one barrier that publishes its inputs (two LDS
    // slots by stage parity: the v3 region, unused here, is the second), the
    // waves' parts of the sweep bound mu (from the previous state, so they
    // are formed at the end of the previous stage) and the previous stage's
    // state-row norms; then the sweeps' stencils and the residual's.
    double *uvs[2] = {uvec, lds_ptr<double>(c, c.off.v3)};
    double xp[RY][CX];
#pragma unroll
    for (int t = 0; t < RY; ++t)
#pragma unroll
        for (int q = 0; q < CX; ++q) xp[t][q] = valid(t, q) ? a.x0[(size_t)b * n + pidx(t, q)] : 0.0;
    // the sweep matrix's row-sum bound for the state after `xs`, this wave's part
    auto mu_part = [&](const double (&xs)[RY][CX]) {
        double m = 0.0;
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q)
                if (valid(t, q)) {
                    const double hk = h * P.k0 * (1.0 + P.k1 * xs[t][q]) * P.c0;
                    m = fmax(m, hk / (1.0 + hk));
                }
        const unsigned long long mb = wave_max64(abits(m), c.lane);
        if (c.lane == 0) nrm[c.w * 4 + 3] = mb;
    };
    if (c.tid < M) uvs[0][c.tid] = a.U[0][(size_t)b * P.N * M + c.tid];
    mu_part(xp);
    for (int i = 0; i < P.N; ++i) {
        const size_t unit = (size_t)b * P.N + i;
        __syncthreads();   // inputs, mu parts and the previous stage's norms are in LDS
        unsigned long long mb = 0;
        for (int ww = 0; ww < c.W; ++ww) mb = umax64(mb, nrm[ww * 4 + 3]);
        const double mu = fmin(1.02 * bits2d(mb), 0.995);
        if (i > 0 && c.tid == 0) {   // provisional: the state rows' norm, completed below
            unsigned long long ax = 0;
            for (int ww = 0; ww < c.W; ++ww) ax = umax64(ax, nrm[ww * 4]);
            a.rst[unit - 1] = ax;
        }
        if (c.Gv == 1) __syncthreads();   // no stencil barrier comes before the slots are rewritten
        const double *uv = uvs[i & 1];
        double Bu[RY][CX], x[RY][CX];
        b_apply<double, CX, RY, LX, LY>(uv, c, Bu);
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q) x[t][q] = xp[t][q];
        double xo[RY][CX], w = 1.0;
        for (int s = 0; s < nsw; ++s) {
            double nb[RY][CX];
            nbsum<double, CX, RY>(x, nb, c);
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) {
                    const double kk = P.k0 * (1.0 + P.k1 * x[t][q]);
                    double v = (xp[t][q] + h * kk * nb[t][q] + h * Bu[t][q]) /
                               (1.0 + h * kk * P.c0);
                    v = valid(t, q) ? v : 0.0;
                    if (s > 0) v = xo[t][q] + w * (v - xo[t][q]);
                    xo[t][q] = x[t][q];
                    x[t][q] = v;
                }
            w = cheb_next(s, w, mu * mu);
        }
        {   // state rows of the built start: K^x_i = x_{i-1} - x_i + h f(u_i, x_i)
            double nb[RY][CX];
            nbsum<double, CX, RY>(x, nb, c);
            unsigned long long mx = 0;
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q)
                    if (valid(t, q)) {
                        const double kk = P.k0 * (1.0 + P.k1 * x[t][q]);
                        const double kx = xp[t][q] - x[t][q] +
                                          h * (kk * (nb[t][q] - P.c0 * x[t][q]) + Bu[t][q]);
                        mx = umax64(mx, abits(kx));
                    }
            mx = wave_max64(mx, c.lane);
            if (c.lane == 0) nrm[c.w * 4] = mx;
        }
        // the next stage's inputs (the slot its predecessor read two stages
        // ago) and its mu parts
        if (i + 1 < P.N) {
            if (c.tid < M) uvs[(i + 1) & 1][c.tid] = a.U[0][(unit + 1) * M + c.tid];
            mu_part(x);
        }
        double *Xo = a.X[0] + unit * n;
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q) {
                if (valid(t, q)) Xo[pidx(t, q)] = x[t][q];
                xp[t][q] = x[t][q];
            }
    }
    __syncthreads();
    if (c.tid == 0) {   // the last stage's state-row norm
        unsigned long long ax = 0;
        for (int ww = 0; ww < c.W; ++ww) ax = umax64(ax, nrm[ww * 4]);
        a.rst[(size_t)b * P.N + P.N - 1] = ax;
    }
    // ---- costates, backward in the horizon
    double ln[RY][CX];
#pragma unroll
    for (int t = 0; t < RY; ++t)
#pragma unroll
        for (int q = 0; q < CX; ++q) ln[t][q] = 0.0;
    for (int i = P.N - 1; i >= 0; --i) {
        const size_t unit = (size_t)b * P.N + i;
        const double *Xi = a.X[0] + unit * n;
        double *Li = a.LAM[0] + unit * n;
        const double *Xr = a.xref + (size_t)b * a.xref_inst_stride + (size_t)i * a.xref_stage_stride;
        double x[RY][CX], Lx[RY][CX], lam[RY][CX];   // the costate sweeps start from zero
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q) {
                x[t][q] = valid(t, q) ? Xi[pidx(t, q)] : 0.0;
                lam[t][q] = 0.0;
            }
        nbsum<double, CX, RY>(x, Lx, c);
        double cc[RY][CX], invd[RY][CX], cpk[RY][CX];
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q) {
                Lx[t][q] -= P.c0 * x[t][q];
                const double kk = P.k0 * (1.0 + P.k1 * x[t][q]);
                const double d = -1.0 - h * kk * P.c0 + h * kp * Lx[t][q];
                invd[t][q] = valid(t, q) ? 1.0 / d : 0.0;
                cpk[t][q] = h * kk;
                const double xr = valid(t, q) ? Xr[pidx(t, q)] : 0.0;
                cc[t][q] = valid(t, q) ? -(ln[t][q] + h * P.q * (x[t][q] - xr)) : 0.0;
            }
        double mu = 0.0;
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q) mu = fmax(mu, P.c0 * cpk[t][q] * fabs(invd[t][q]));
        mu = fmin(1.02 * block_max_nonneg(mu, c, nrm), 0.995);
        double lo[RY][CX], w = 1.0;
        for (int s = 0; s < nswl; ++s) {
            double z[RY][CX], nb[RY][CX];
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) z[t][q] = cpk[t][q] * lam[t][q];
            nbsum<double, CX, RY>(z, nb, c);
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) {
                    double v = (cc[t][q] - nb[t][q]) * invd[t][q];
                    if (s > 0) v = lo[t][q] + w * (v - lo[t][q]);
                    lo[t][q] = lam[t][q];
                    lam[t][q] = v;
                }
            w = cheb_next(s, w, mu * mu);
        }
        {   // costate and input rows of the built start, then the stage norms
            double z[RY][CX], nb[RY][CX];
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) z[t][q] = cpk[t][q] * lam[t][q];
            nbsum<double, CX, RY>(z, nb, c);
            unsigned long long ml = 0, mu = 0;
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q)
                    if (valid(t, q)) {
                        // K^lam_i = -(cc - diag(F_x^T) lam - offdiag(F_x^T) lam)
                        const double kk = P.k0 * (1.0 + P.k1 * x[t][q]);
                        const double d = -1.0 - h * kk * P.c0 + h * kp * Lx[t][q];
                        ml = umax64(ml, abits(cc[t][q] - d * lam[t][q] - nb[t][q]));
                    }
            const double bt = bt_reduce<double, CX, RY, LX, LY>(lam, c, M);
            if (c.tid < M) {   // K^u_i = h (r u_i + grad Phi(u_i) + B^T lam_i)
                const double u = a.U[0][unit * M + c.tid];
                double bg = 0.0;
                if (P.tau > 0.0) bg = -P.tau / (u - P.ulo) + P.tau / (P.uhi - u);
                mu = abits(h * (P.r * u + bg + bt));
            }
            ml = wave_max64(ml, c.lane);
            mu = wave_max64(mu, c.lane);
            if (c.lane == 0) { nrm[c.w * 4 + 1] = ml; nrm[c.w * 4 + 2] = mu; }
            __syncthreads();
            if (c.tid == 0) {
                unsigned long long al = 0, au = 0;
                for (int ww = 0; ww < c.W; ++ww) {
                    al = umax64(al, nrm[ww * 4 + 1]);
                    au = umax64(au, nrm[ww * 4 + 2]);
                }
                const unsigned long long ax = a.rst[unit];
                const double dx_ = bits2d(ax), dl_ = bits2d(al), du_ = bits2d(au);
                double rp = fmax(fmax(dx_, du_), dl_);
                double rs = fmax(fmax(dx_, du_ / (h * P.r)), dl_ / h);
                if (ax >= 0x7FF0000000000000ull || al >= 0x7FF0000000000000ull ||
                    au >= 0x7FF0000000000000ull)
                    rs = rp = __longlong_as_double(0x7FF8000000000000ll);
                a.rst[unit] = abits(rs);
                a.pst[unit] = abits(rp);
            }
        }
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q) {
                if (valid(t, q)) Li[pidx(t, q)] = lam[t][q];
                ln[t][q] = lam[t][q];
            }
    }
}

// Fallback between two starts, per instance: keep buffer 0's start unless its
// residual (slot 0) is non-finite or larger than that of the start in buffer
// 1 (slot 1). start_used[b] = used_if_kept, or 0 (the buffer-1 start). With
// res_first_stage, slot 1 holds the buffer-1 start's stage-0 residual only
// (a cold start with one reference for all stages has the same residual at
// every stage).
__global__ void k_choose_flags(const IterArgs a, int *start_used, int used_if_kept)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.units) return;
    const size_t N = a.P.N;
    unsigned long long mw = 0, mc = 0;
    for (size_t i = 0; i < N; ++i) {
        mw = umax64(mw, a.rst[(size_t)b * N + i]);
        if (!a.res_first_stage || i == 0) mc = umax64(mc, a.rst[((size_t)a.B + b) * N + i]);
    }
    start_used[b] = (bits2d(mw) <= bits2d(mc)) ? used_if_kept : 0;
}

// Write the cold start (x_i = x0 with its zero padding, u_i = 0, lambda_i =
// 0) into buffer 0 for the instances that fell back.
__global__ void k_choose_copy(const IterArgs a, const int *start_used)
{
    // one workgroup per (instance, stage); instances that keep their start
    // return at once
    const size_t np = a.P.n, N = a.P.N, m = a.P.m;
    const size_t unit = blockIdx.x, b = unit / N;
    if (b >= (size_t)a.units || start_used[b] != 0) return;
    for (size_t p = threadIdx.x; p < np; p += blockDim.x) {
        a.X[0][unit * np + p] = a.x0[b * np + p];
        a.LAM[0][unit * np + p] = 0.0;
    }
    for (size_t j = threadIdx.x; j < m; j += blockDim.x) a.U[0][unit * m + j] = 0.0;
}

// Advances the device kernel base index after a captured sequence of `len`
// iteration launches (whose own indices come from their kofs arguments).
__global__ void k_advance(int *ctr, int len)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctr[0] += len;
}

// S^0 into buffer 0 in the padded stage layout (row stride sx, zero
// padding): cold (x_i = x0, u_i = 0, lam_i = 0) or the warm start given in
// the dense [count][N][n] layout.
__global__ void k_init(const InitArgs a)
{
    const size_t np = (size_t)a.nsy * a.sx;             // padded points per stage
    const size_t nst = a.nst > 0 ? a.nst : a.N;        // stages written per instance
    const size_t nN = (size_t)a.count * nst * np;
    const size_t mN = (size_t)a.count * nst * a.m;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    // padding only, and the rows have none: nothing to write here
    const size_t nNw = a.pad_only && a.sx == a.nsx ? 0 : nN;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < nNw; t += stride) {
        const size_t us = t / np, p = t % np;
        const size_t b = us / nst, unit = b * a.N + us % nst;
        const int row = (int)(p / a.sx), col = (int)(p % a.sx);
        if (a.pad_only && col < a.nsx) continue;
        double x = 0.0, l = 0.0;
        if (col < a.nsx) {
            const size_t dense = unit * (size_t)a.nsx * a.nsy + (size_t)row * a.nsx + col;
            x = a.wx ? a.wx[dense] : a.x0[b * np + p];
            l = a.wl ? a.wl[dense] : 0.0;
        }
        a.X[unit * np + p] = x;
        a.LAM[unit * np + p] = l;
    }
    // with an input box the method starts from a strictly feasible S^0
    // (Sec. 4.2): given inputs are clipped to the box shrunk by 0.5 % of its
    // width at each end (NaN stays NaN, so the residual test still rejects it)
    const double marg = 0.005 * (a.uhi - a.ulo);
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < mN; t += stride) {
        const size_t b = t / (nst * a.m), r = t % (nst * a.m);
        const size_t e = b * a.N * a.m + r;
        double u = a.wu ? a.wu[e] : 0.0;
        if (a.project && a.wu) {
            if (u < a.ulo + marg) u = a.ulo + marg;
            if (u > a.uhi - marg) u = a.uhi - marg;
        }
        a.U[e] = u;
    }
    if (a.trajectory_only) return;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)a.count;
         t += stride) {
        InstState s;
        s.status = kActive; s.mode = a.mode; s.e = 0; s.j = 0; s.pending = 0; s.f32 = 0;
        s.eonly = s.pad = 0;
        a.st[t] = s;
        a.st[a.B + t] = s;
        a.iters[t] = 0;
        if (a.du) { a.du[2 * t] = 0; a.du[2 * t + 1] = 0; }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctr[0] = 0;
        a.ctr[2] = 0;
        a.ctr[3] = a.mode == kModeFp32 ? a.count : 0;
    }
}

// Dense rows [rows][nsx] -> padded rows [rows][sx] (zero padding).
__global__ void k_pad(const double *src, double *dst, long long rows, int nsx, int sx)
{
    const size_t tot = (size_t)rows * sx, stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
        const size_t r = t / sx;
        const int col = (int)(t % sx);
        dst[t] = col < nsx ? src[r * nsx + col] : 0.0;
    }
}

// Returned iterates to the caller's dense outputs: unit (instance, stage)
// blockIdx.y (strided), its points over blockIdx.x; each instance reads the
// buffer that holds its returned iterate (iters[b] & 1).
__global__ void k_output(const OutArgs a)
{
    const int units = a.count * a.N, n = a.nsx * a.nsy;
    const size_t np = (size_t)a.nsy * a.sx;
    for (int unit = blockIdx.y; unit < units; unit += gridDim.y) {
        const int buf = a.iters[unit / a.N] & 1;
        const double *X = a.X[buf] + unit * np, *L = a.LAM[buf] + unit * np;
        double *ox = a.ox + (size_t)unit * n, *ol = a.ol + (size_t)unit * n;
        if (a.vec) {   // pairs of columns of one row
            for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n / 2; t += gridDim.x * blockDim.x) {
                const int p = 2 * t, row = p / a.nsx;
                const size_t src = (size_t)row * a.sx + (p - row * a.nsx);
                *reinterpret_cast<double2 *>(ox + p) = *reinterpret_cast<const double2 *>(X + src);
                *reinterpret_cast<double2 *>(ol + p) = *reinterpret_cast<const double2 *>(L + src);
            }
        } else {
            for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
                const int row = p / a.nsx;
                const size_t src = (size_t)row * a.sx + (p - row * a.nsx);
                ox[p] = X[src];
                ol[p] = L[src];
            }
        }
        if (blockIdx.x == 0)
            for (int j = threadIdx.x; j < a.m; j += blockDim.x)
                a.ou[(size_t)unit * a.m + j] = a.U[buf][(size_t)unit * a.m + j];
    }
}

// ------------------------------------------------------ instantiation table

// Tile shapes: CX columns x RY rows per lane, at most WB waves per workgroup
// (WB * 4 * RY >= 64 rows, 96 for CX = 6). The first entry per (precision, CX)
// is the default; the others are alternatives for the tile autotuner.
#define NMPC_TILE(P, CX_, RY_, WB_)                                                 \
    if (prec == P && cx == CX_ && (ry == 0 || ry == RY_) && lx == LX_ && ly == LY_) { \
        cfg->cx = CX_; cfg->rows = RY_; cfg->max_waves = WB_;                       \
        return (const void *)&k_iterate<P, CX_, RY_, WB_, NMPC_OCC(WB_), LX_, LY_>;  \
    }
// waves per SIMD requested from the register allocator: two workgroups of up
// to 8 waves per CU
#define NMPC_OCC(WB_) 2
#define NMPC_LATTICE()                                                              \
    NMPC_TILE(kModeFp32, 1, 4, 4) NMPC_TILE(kModeFp32, 1, 8, 2)                     \
    NMPC_TILE(kModeFp32, 2, 4, 4) NMPC_TILE(kModeFp32, 2, 8, 2)                     \
    NMPC_TILE(kModeFp32, 3, 4, 4) NMPC_TILE(kModeFp32, 3, 2, 8)                     \
    NMPC_TILE(kModeFp32, 4, 4, 4) NMPC_TILE(kModeFp32, 4, 2, 8)                     \
    NMPC_TILE(kModeFp32, 6, 3, 8)                                                  \
    NMPC_TILE(kModeFp64, 1, 4, 4) NMPC_TILE(kModeFp64, 2, 2, 8)                     \
    NMPC_TILE(kModeFp64, 2, 4, 4) NMPC_TILE(kModeFp64, 3, 2, 8)                     \
    NMPC_TILE(kModeFp64, 4, 2, 8)                                                   \
    NMPC_TILE(kModeFp64, 6, 3, 8)

const void *iterate_kernel(int prec, int cx, int ry, int lx, int ly, TileCfg *cfg)
{
#define LX_ 1
#define LY_ 1
    NMPC_LATTICE()
#undef LX_
#undef LY_
#define LX_ 2
#define LY_ 1
    NMPC_LATTICE()
#undef LX_
#undef LY_
#define LX_ 2
#define LY_ 2
    NMPC_LATTICE()
#undef LX_
#undef LY_
#define LX_ 4
#define LY_ 4
    NMPC_LATTICE()
#undef LX_
#undef LY_
    return nullptr;
}
#undef NMPC_LATTICE
#undef NMPC_TILE
#undef NMPC_OCC

#define NMPC_ROLL(CX_, RY_, WB_)                                                    \
    if (cx == CX_ && lx == LX_ && ly == LY_) {                                      \
        cfg->cx = CX_; cfg->rows = RY_; cfg->max_waves = WB_;                       \
        return (const void *)&k_rollout<CX_, RY_, WB_, LX_, LY_>;                    \
    }
#define NMPC_ROLL_LATTICE()                                                         \
    NMPC_ROLL(1, 4, 4) NMPC_ROLL(2, 2, 8) NMPC_ROLL(3, 2, 8) NMPC_ROLL(4, 2, 8)     \
    NMPC_ROLL(6, 3, 8)

const void *rollout_kernel(int cx, int lx, int ly, TileCfg *cfg)
{
#define LX_ 1
#define LY_ 1
    NMPC_ROLL_LATTICE()
#undef LX_
#undef LY_
#define LX_ 2
#define LY_ 1
    NMPC_ROLL_LATTICE()
#undef LX_
#undef LY_
#define LX_ 2
#define LY_ 2
    NMPC_ROLL_LATTICE()
#undef LX_
#undef LY_
#define LX_ 4
#define LY_ 4
    NMPC_ROLL_LATTICE()
#undef LX_
#undef LY_
    return nullptr;
}
#undef NMPC_ROLL_LATTICE
#undef NMPC_ROLL

const void *init_kernel() { return (const void *)&k_init; }
const void *box_apply_kernel() { return (const void *)&k_box_apply; }
const void *choose_flags_kernel() { return (const void *)&k_choose_flags; }
const void *choose_copy_kernel() { return (const void *)&k_choose_copy; }
const void *pad_kernel() { return (const void *)&k_pad; }
const void *advance_kernel() { return (const void *)&k_advance; }
const void *output_kernel() { return (const void *)&k_output; }

}  // namespace nmpc
