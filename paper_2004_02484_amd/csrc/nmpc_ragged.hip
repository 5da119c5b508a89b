// nmpc_ragged.hip -- the upper iteration over a ragged batch:
// instances of different grid sizes and horizons (each instance belongs to a
// problem class with its own grid, horizon, step and input factors).
//
// All classes share the workgroup size; each class gets the tile (CX columns
// x RY rows per lane) that covers its grid with the fewest rows. One upper
// iteration is one launch per tile case present in the batch, all captured in
// the same graph. A case's work list holds one entry per (instance, stage)
// unit of its instances, grouped into eight runs, one per XCD (consecutive
// workgroup ids go to different XCDs), each run balanced by stage-points and
// holding whole instances, so that the x_{i-1} / lambda_{i+1} reads of
// neighbouring stages hit that XCD's L2. The per-instance convergence state
// machine is the one of the batch kernel, with the instance's own horizon.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "nmpc_device.h"
#include "nmpc_stage.h"

namespace nmpc {

constexpr int kRgLx = 4, kRgLy = 4;
constexpr int kRgCx[5] = {1, 2, 3, 4, 6};

// Rows covered by a tile of RY rows per lane with WB waves: 4 * WB * RY. A
// case is instantiated only where it is the smallest cover of some grid
// height <= 96 and has at most 18 (8 waves) or 12 (12, 16 waves) points per
// lane, so that its registers fit what WB waves leave a lane (512 / (WB / 4)
// VGPRs, at most 256); the autotuner weighs tile size against occupancy.
__host__ __device__ constexpr int rg_max_points(int wb) { return wb <= 8 ? 18 : 12; }
template <int WB, int CX, int RY>
constexpr bool rg_case() { return 4 * WB * (RY - 1) < 96 && CX * RY <= rg_max_points(WB); }

// One launch per tile case present in the batch: the units of the instances
// whose class takes this tile (CX x RY per lane), eight XCD runs of per_xcd
// units each. Every case is its own kernel, so each gets the register
// allocation of its tile and no call boundary.
template <int PREC, int WB, int CX, int RY>
__global__ void __launch_bounds__(kWave * WB, 1) k_iterate_rg(const IterArgs a, const RgArgs r)
{
    using T = typename std::conditional<PREC == kModeFp32, float, double>::type;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int k = a.residual_only ? 0 : *(volatile const int *)(a.ctr) + a.kofs;
    const int bid = blockIdx.x;
    const int unit = (bid & 7) * a.per_xcd + (bid >> 3);
    if (unit >= a.units) return;
    const int2 bi = r.umap[unit];
    if (bi.x < 0) return;
    const int b = bi.x, i = bi.y;
    const RgClass &cl = r.cls[r.icls[b]];
    Ctx c;
    c.lds = lds_raw;
    tile_setup<T, CX, RY, kRgLx, kRgLy>(c, cl.P);
    const int N = cl.P.N;
    const long long us = r.ustart[b];
    Decision d;
    if (a.residual_only) {
        d.work = true; d.j = 0; d.slot = a.res_slot; d.eval_only = false; d.redo = false;
    } else {
        d = decide<PREC>(a, c, b, i, k, N, us);
    }
    if (!d.work) return;
    StageLoc v = jacobi_loc(d.j & 1);
    v.tgx = cl.gx;   // tables loaded after the stage's loads are issued
    v.tgy = cl.gy;
    v.defer_norms = true;
    v.so = r.soff[b];
    v.uo = r.uoff[b];
    v.xo = r.xoff[b];
    v.xro = r.xoff[b];
    v.res_at = (long long)d.slot * a.rslot + us + i;
    v.res_only = d.eval_only;
    if (d.redo && a.du) v.du_at = b;
    if (cl.P.tau > 0.0 && !a.residual_only && !d.eval_only) {   // input box: record the limit
        v.box_at = us + i;
        if (i == 0 && c.tid == 0) a.aupd[b] = k + 1;   // this launch updates b
    }
    v.i = i;
    v.last = i == N - 1;
    unsigned long long acc[2] = {0, 0};
    stage_body<T, CX, RY, kRgLx, kRgLy>(a, cl.P, v, c, acc);
}

// Dense inputs [count][n_b] (packed) -> padded rows (stride sx of the
// instance's class, zero padding). One workgroup per instance.
__global__ void k_rg_pad(const RgArgs r, const double *src, double *dst)
{
    const int b = blockIdx.x;
    if (b >= r.count) return;
    const RgClass &cl = r.cls[r.icls[b]];
    const int nsx = cl.P.nsx, sx = cl.sx, tot = cl.P.nsy * sx;
    const double *s = src + r.dxoff[b];
    double *d = dst + r.xoff[b];
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        const int row = t / sx, col = t % sx;
        d[t] = col < nsx ? s[row * nsx + col] : 0.0;
    }
}

// S^0 of each instance into buffer 0: cold (x_i = x0, u_i = 0, lambda_i = 0)
// or the given dense start; iteration state reset. One workgroup per instance.
__global__ void k_rg_init(const IterArgs a, const RgArgs r, int mode, const double *wx,
                          const double *wu, const double *wl)
{
    const int b = blockIdx.x;
    if (b >= r.count) return;
    const RgClass &cl = r.cls[r.icls[b]];
    const int nsx = cl.P.nsx, sx = cl.sx, np = cl.P.n, N = cl.P.N, m = cl.P.m;
    const int nd = nsx * cl.P.nsy;
    const double *x0 = a.x0 + r.xoff[b];
    double *X = a.X[0] + r.soff[b];
    double *L = a.LAM[0] + r.soff[b];
    double *U = a.U[0] + r.uoff[b];
    const long long ds = r.dsoff[b];
    for (long long t = threadIdx.x; t < (long long)N * np; t += blockDim.x) {
        const int i = (int)(t / np), p = (int)(t % np);
        const int row = p / sx, col = p % sx;
        double x = 0.0, l = 0.0;
        if (col < nsx) {
            const long long dense = ds + (long long)i * nd + row * nsx + col;
            x = wx ? wx[dense] : x0[p];
            l = wl ? wl[dense] : 0.0;
        }
        X[t] = x;
        L[t] = l;
    }
    // with an input box the start is strictly feasible (Sec. 4.2): given inputs
    // are clipped to the box shrunk by 0.5 % of its width at each end
    const double ulo = cl.P.ulo, uhi = cl.P.uhi, marg = 0.005 * (uhi - ulo);
    for (int t = threadIdx.x; t < N * m; t += blockDim.x) {
        double u = wu ? wu[r.uoff[b] + t] : 0.0;
        if (wu && cl.P.tau > 0.0) {
            if (u < ulo + marg) u = ulo + marg;
            if (u > uhi - marg) u = uhi - marg;
        }
        U[t] = u;
    }
    if (threadIdx.x == 0) {
        InstState s;
        s.status = kActive; s.mode = mode; s.e = 0; s.j = 0; s.pending = 0; s.f32 = 0;
        s.eonly = s.pad = 0;
        a.st[b] = s;
        a.st[a.B + b] = s;
        a.iters[b] = 0;
        if (a.du) { a.du[2 * b] = 0; a.du[2 * b + 1] = 0; }
    }
    if (b == 0 && threadIdx.x == 0) {
        a.ctr[0] = 0;
        a.ctr[2] = 0;
        a.ctr[3] = mode == kModeFp32 ? r.count : 0;
    }
}

// Each instance's returned iterate (buffer iters[b] & 1) to the dense packed
// outputs. One workgroup per instance.
__global__ void k_rg_output(const IterArgs a, const RgArgs r, double *ox, double *ou, double *ol)
{
    const int b = blockIdx.x;
    if (b >= r.count) return;
    const RgClass &cl = r.cls[r.icls[b]];
    const int nsx = cl.P.nsx, sx = cl.sx, np = cl.P.n, N = cl.P.N, m = cl.P.m;
    const int nd = nsx * cl.P.nsy;
    const int buf = a.iters[b] & 1;
    const double *X = a.X[buf] + r.soff[b];
    const double *L = a.LAM[buf] + r.soff[b];
    const double *U = a.U[buf] + r.uoff[b];
    const long long ds = r.dsoff[b];
    for (long long t = threadIdx.x; t < (long long)N * nd; t += blockDim.x) {
        const int i = (int)(t / nd), p = (int)(t % nd);
        const long long src = (long long)i * np + (p / nsx) * sx + p % nsx;
        ox[ds + t] = X[src];
        ol[ds + t] = L[src];
    }
    for (int t = threadIdx.x; t < N * m; t += blockDim.x) ou[r.uoff[b] + t] = U[t];
}

template <int PREC, int WB>
const void *rg_kernel(int tcase)
{
#define NMPC_RG_CASE(CI, RY)                                                       \
    case 3 * CI + RY - 1:                                                           \
        if constexpr (rg_case<WB, kRgCx[CI], RY>())                                 \
            return (const void *)&k_iterate_rg<PREC, WB, kRgCx[CI], RY>;             \
        return nullptr;
    switch (tcase) {
        NMPC_RG_CASE(0, 1) NMPC_RG_CASE(0, 2) NMPC_RG_CASE(0, 3)
        NMPC_RG_CASE(1, 1) NMPC_RG_CASE(1, 2) NMPC_RG_CASE(1, 3)
        NMPC_RG_CASE(2, 1) NMPC_RG_CASE(2, 2) NMPC_RG_CASE(2, 3)
        NMPC_RG_CASE(3, 1) NMPC_RG_CASE(3, 2) NMPC_RG_CASE(3, 3)
        NMPC_RG_CASE(4, 1) NMPC_RG_CASE(4, 2) NMPC_RG_CASE(4, 3)
    default: return nullptr;
    }
#undef NMPC_RG_CASE
}

const void *ragged_iterate_kernel(int prec, int waves, int tcase)
{
    if (prec == kModeFp32) {
        if (waves == 8) return rg_kernel<kModeFp32, 8>(tcase);
        if (waves == 12) return rg_kernel<kModeFp32, 12>(tcase);
        if (waves == 16) return rg_kernel<kModeFp32, 16>(tcase);
    } else {
        if (waves == 8) return rg_kernel<kModeFp64, 8>(tcase);
        if (waves == 12) return rg_kernel<kModeFp64, 12>(tcase);
        if (waves == 16) return rg_kernel<kModeFp64, 16>(tcase);
    }
    return nullptr;
}

int ragged_tile(int nsx, int nsy, int waves, int *cx, int *ry)
{
    int ci = -1;
    for (int q = 0; q < 5; ++q)
        if (16 * kRgCx[q] >= nsx) { ci = q; break; }
    if (ci < 0 || nsy < 1 || nsx < 1) return -1;
    const int rows = 4 * waves;
    const int r_ = (nsy + rows - 1) / rows;
    if (r_ > 3 || 4 * waves * (r_ - 1) >= 96 || kRgCx[ci] * r_ > rg_max_points(waves)) return -1;
    if (cx) *cx = kRgCx[ci];
    if (ry) *ry = r_;
    return 3 * ci + r_ - 1;
}

// Input box after an iteration launch of one tile case (the units of its
// work list): the fraction-to-the-boundary rule (eq. eq_alphamax) with alpha
// global over an instance's stages, as for the batch kernel. Instances that
// did not update in this launch, have no box, or have alpha = 1 return at once.
__global__ void __launch_bounds__(256) k_rg_box_apply(const IterArgs a, const RgArgs r)
{
    __shared__ double red[256];
    const int k = *(volatile const int *)(a.ctr) + a.kofs;
    const int bid = blockIdx.x;
    const int unit = (bid & 7) * a.per_xcd + (bid >> 3);
    if (unit >= a.units) return;
    const int2 bi = r.umap[unit];
    if (bi.x < 0) return;
    const int b = bi.x, i = bi.y;
    const RgClass &cl = r.cls[r.icls[b]];
    if (!(cl.P.tau > 0.0) || a.aupd[b] != k + 1) return;
    const int N = cl.P.N, n = cl.P.n, M = cl.P.m;
    const long long us = r.ustart[b];
    double l = 1.0;
    for (int t = threadIdx.x; t < N; t += blockDim.x) l = fmin(l, a.apart[us + t]);
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const double alpha = red[0];
    if (!(alpha < 1.0)) return;
    const int src = a.st[((k + 1) & 1) * a.B + b].j & 1, dst = src ^ 1;
    const size_t so = (size_t)r.soff[b] + (size_t)i * n, uo = (size_t)r.uoff[b] + (size_t)i * M;
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
        const double xs = a.X[src][so + p], ls = a.LAM[src][so + p];
        a.X[dst][so + p] = xs + alpha * (a.X[dst][so + p] - xs);
        a.LAM[dst][so + p] = ls + alpha * (a.LAM[dst][so + p] - ls);
    }
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const double us_ = a.U[src][uo + j];
        a.U[dst][uo + j] = us_ + alpha * (a.U[dst][uo + j] - us_);
    }
}

const void *ragged_pad_kernel() { return (const void *)&k_rg_pad; }
const void *ragged_box_apply_kernel() { return (const void *)&k_rg_box_apply; }
const void *ragged_init_kernel() { return (const void *)&k_rg_init; }
const void *ragged_output_kernel() { return (const void *)&k_rg_output; }

}  // namespace nmpc
