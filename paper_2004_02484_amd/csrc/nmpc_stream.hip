// nmpc_stream.hip -- streaming kernels of the Jacobi upper iteration for grids
// whose stage does not fit one workgroup (e.g. 256 x 256): each step of the
// stage algebra is a pass over all stages of the batch, with per-unit partial
// reductions combined by small per-stage kernels.
//
// One upper iteration (eq. 1st_jacobi, alpha = 1), per instance and stage i:
//   res      KKT rows K^x, K^lambda (FP64), stage coefficients, unit partials
//            of the norms and of B^T lambda
//   stage    K^u = h (r u + B^T lambda), the stage's norms, v3 = 0
//   decide   per-instance state machine (test, phases, max_iter)
//   Schur iterations (Sec. 5.2):  y5 = JacF(h B v3 - b1); c' = -b2 - A_xx y5;
//            y4 = JacFT(c'), partials of B^T y4; v3 = (K^u + h B^T y4)/A_uu
//   final:   y5 = JacF(b1 - h B v3); y4 = JacFT(b2 - A_xx y5);
//            S^{k+1} = S^k - (y5, v3, y4)
// With two point-Jacobi sweeps per solve (the default) the residual pass and
// each Schur step / final block are single marching-strip passes (one wave
// per strip of columns and block of rows, stencils in registers and lane
// shifts, no LDS stencils or barriers): the residual pass also takes the
// first Schur step (v3 = 0 needs no stage reduction), each later pass forms
// its v3 from the previous step's unit partials, and the final block forms
// the stage coefficients from the x and lambda it reads for the update. Other
// sweep counts use row-block passes with LDS-staged stencils: a solve is one
// pass for its first two sweeps and one per further sweep.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "nmpc_device.h"

namespace nmpc {

namespace {

__device__ __forceinline__ unsigned long long sabits(double v)
{
    return (unsigned long long)__double_as_longlong(fabs(v));
}
__device__ __forceinline__ double sbits2d(unsigned long long b)
{
    return __longlong_as_double((long long)b);
}
__device__ __forceinline__ unsigned long long sumax(unsigned long long a, unsigned long long b)
{
    return a > b ? a : b;
}

// Row-block unit of a pass: one workgroup of 4 waves per block of kRows grid
// rows of one stage, XCD-aware order (each XCD a contiguous run of blocks, so
// a stage's neighbouring blocks and stages share that XCD's L2). Inputs of a
// stencil are staged in LDS for the block's rows plus one halo row above and
// below (zero outside the grid: the Dirichlet values); wave w computes rows
// w, w + 4, ... of the block, lanes walk the columns, so per-row reductions
// are wave reductions without barriers.
constexpr int kRows = kStreamRows;

struct Block {
    int b, i, iy0;
    bool ok;
};

__device__ __forceinline__ Block row_block(const StreamArgs &a)
{
    Block r{};
    const int bid = blockIdx.x;
    const long long unit = (long long)(bid & 7) * a.per_xcd + (bid >> 3);
    if (unit >= a.units) { r.ok = false; return r; }
    const int nblk = (a.P.nsy + kRows - 1) / kRows;
    r.iy0 = (int)(unit % nblk) * kRows;
    const long long bi = unit / nblk;
    r.i = (int)(bi % a.P.N);
    r.b = (int)(bi / a.P.N);
    r.ok = r.b < a.count;
    return r;
}

// Work flag for the residual pass: the instance is active in this phase.
template <int PREC>
__device__ __forceinline__ bool evaluating(const StreamArgs &a, int b)
{
    const InstState &s = a.st[b];
    if (s.status != kActive) return false;
    return PREC == kModeFp32 ? s.mode == kModeFp32 : s.mode != kModeFp32;
}

// Visit the staged rows iy0 - 1 .. iy0 + kRows of a block: body(e, iy, ix,
// inside, cv) for LDS index e = rr * nsx + ix, with inside false outside the
// grid (the staged value is then the Dirichlet zero). Threads own columns
// (ix = thread, thread + 256, ...; g thread groups share the rows when the row
// is narrower than the workgroup) and walk the rows, so the addresses need no
// division per element and a value a column needs in every row (cv = col(ix),
// e.g. the column sums of B v) is loaded once. The caller synchronizes.
template <typename COL, typename F>
__device__ __forceinline__ void for_staged(const DevProblem &P, int iy0, COL col, F body)
{
    const int nsx = P.nsx;
    const int g = nsx >= (int)blockDim.x ? 1 : (int)blockDim.x / nsx;
    const int r0 = g == 1 ? 0 : (int)threadIdx.x / nsx;
    const int c0 = (int)threadIdx.x - r0 * nsx;
    if (r0 >= g) return;
    for (int ix = c0; ix < nsx; ix += g == 1 ? (int)blockDim.x : nsx) {
        auto cv = col(ix);
#pragma unroll 2
        for (int rr = r0; rr < kRows + 2; rr += g) {
            const int iy = iy0 + rr - 1;
            body(rr * nsx + ix, iy, ix, iy >= 0 && iy < P.nsy, cv);
        }
    }
}

struct NoCol {};
__device__ __forceinline__ NoCol no_col(int) { return NoCol{}; }

// Stage f(iy, ix) for the block's rows and halo rows into lds [(kRows + 2)][nsx]
// and synchronize.
template <typename V, typename F>
__device__ __forceinline__ void stage_rows(V *lds, const DevProblem &P, int iy0, F f)
{
    for_staged(P, iy0, no_col, [&](int e, int iy, int ix, bool in, NoCol) {
        lds[e] = in ? f(iy, ix) : V(0);
    });
    __syncthreads();
}

// The ly column sums sc[bb][ix] of B v for one column (registers; the loops
// over the lattice rows are unrolled to kMaxLy so the array stays in VGPRs).
struct BCol {
    double s[kMaxLy];
};

// Neighbour sum of a staged array at block row rr (0-based), column ix.
template <typename V>
__device__ __forceinline__ V lds_nb(const V *lds, int nsx, int rr, int ix, V ax, V ay)
{
    const V *row = lds + (rr + 1) * nsx;
    const V l = ix > 0 ? row[ix - 1] : V(0), r = ix + 1 < nsx ? row[ix + 1] : V(0);
    return ax * (l + r) + ay * (row[ix - nsx] + row[ix + nsx]);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    return v;
}
__device__ __forceinline__ unsigned long long wave_umax(unsigned long long v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = sumax(v, __shfl_xor(v, m, kWave));
    return v;
}

// Wave-wide lane shifts (DPP wave_shl:1 / wave_shr:1): the value of the
// next / previous lane, zero at the wave's end / start.
template <typename T>
__device__ __forceinline__ T wshl(T v);   // lane l gets lane l + 1 (0 at the end)
template <typename T>
__device__ __forceinline__ T wshr(T v);   // lane l gets lane l - 1 (0 at the start)
template <>
__device__ __forceinline__ float wshl<float>(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
template <>
__device__ __forceinline__ float wshr<float>(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
template <>
__device__ __forceinline__ double wshl<double>(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x130, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <>
__device__ __forceinline__ double wshr<double>(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Own rows of the block for this wave: rows iy0 + w, iy0 + w + 4, ... < nsy;
// body(rr, iy) for each. Lanes then walk the columns inside body.
template <typename F>
__device__ __forceinline__ void own_rows(const DevProblem &P, int iy0, F body)
{
    const int w = threadIdx.x / kWave;
    for (int rr = w; rr < kRows && iy0 + rr < P.nsy; rr += (int)(blockDim.x / kWave)) body(rr, iy0 + rr);
}

}  // namespace

// sc[b][i][bb][ix] = sum_a gx[a][ix] v[b][i][bb * lx + a]  (which = 0: U of
// the current iterate, for the instances this graph evaluates; 1: v3, for
// those it steps); (B v)_p = sum_bb gy[bb][iy] sc[bb][ix]. One workgroup per
// (instance, stage). Used by the multi-pass lower layer (more than two sweeps
// per solve); the residual and fused passes form these sums themselves.
template <int PREC>
__global__ void k_st_bsep(const StreamArgs a, int which)
{
    const int bi = blockIdx.x;
    if (bi >= a.count * a.P.N) return;
    const int b = bi / a.P.N;
    if (which == 0 ? !evaluating<PREC>(a, b) : a.work[b] == 0) return;
    const int m = a.P.m, lx = a.P.lx, nsx = a.P.nsx;
    const double *v = which == 0 ? a.U[a.st[b].j & 1] + (size_t)bi * m : a.v3 + (size_t)bi * m;
    double *sc = a.sc + (size_t)bi * a.P.ly * nsx;
    for (int t = threadIdx.x; t < a.P.ly * nsx; t += blockDim.x) {
        const int bb = t / nsx, ix = t % nsx;
        double s = 0.0;
        for (int aa = 0; aa < lx; ++aa) s += a.gx[aa * nsx + ix] * v[bb * lx + aa];
        sc[t] = s;
    }
}

__device__ __forceinline__ double bsep_at(const StreamArgs &a, size_t bi, int iy, int ix)
{
    const double *sc = a.sc + bi * a.P.ly * a.P.nsx;
    double s = 0.0;
    for (int bb = 0; bb < a.P.ly; ++bb) s += a.gy[bb * a.P.nsy + iy] * sc[bb * a.P.nsx + ix];
    return s;
}

__device__ __forceinline__ BCol bsep_col(const StreamArgs &a, size_t bi, int ix)
{
    const double *sc = a.sc + bi * a.P.ly * a.P.nsx;
    BCol c;
#pragma unroll
    for (int bb = 0; bb < kMaxLy; ++bb) c.s[bb] = bb < a.P.ly ? sc[bb * a.P.nsx + ix] : 0.0;
    return c;
}

__device__ __forceinline__ double bsep_row(const StreamArgs &a, const BCol &c, int iy)
{
    double s = 0.0;
#pragma unroll
    for (int bb = 0; bb < kMaxLy; ++bb)
        if (bb < a.P.ly) s += a.gy[bb * a.P.nsy + iy] * c.s[bb];
    return s;
}

// 1 / d for the lower layer (hardware reciprocal in FP32, see the fused kernel).
template <typename T>
__device__ __forceinline__ T st_recip(double d);
template <>
__device__ __forceinline__ float st_recip<float>(double d) { return __builtin_amdgcn_rcpf(float(d)); }
template <>
__device__ __forceinline__ double st_recip<double>(double d) { return 1.0 / d; }

// KKT rows of S^j (FP64), the lower layer's right-hand sides and
// coefficients (stored in T) and the unit partials of the stage norms and of
// B^T lambda. Units as in the lower-layer pass: one wave per strip of 56
// owned columns and kLowerRows rows, each lane marching down its column from
// one row above the block to one below; x and g = k(x) lambda of the row
// above, the row and the row below stay in registers, horizontal neighbours
// come from the adjacent lanes. Rows are loaded PFR rows ahead into a
// register ring.
template <typename T>
__global__ void __launch_bounds__(256, 3) k_st_res(const StreamArgs a)
{
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const long long g = (long long)(blockIdx.x & 7) * a.lper_xcd + (blockIdx.x >> 3);
    const long long unit = g * (blockDim.x / kWave) + wv;
    if (unit >= a.lunits) return;
    const int sp = (int)(unit % a.nstrip);
    const long long t1 = unit / a.nstrip;
    const int rb = (int)(t1 % a.nrb);
    const long long bi = t1 / a.nrb;
    const int b = (int)(bi / a.P.N), i = (int)(bi % a.P.N);
    constexpr int PREC = std::is_same<T, float>::value ? kModeFp32 : kModeFp64;
    if (!evaluating<PREC>(a, b)) return;
    const DevProblem &P = a.P;
    const int nsx = P.nsx, nsy = P.nsy, n = nsx * nsy;
    const int ix = sp * kLowerCols - kLowerHaloX + lane;
    const bool col_in = ix >= 0 && ix < nsx;
    const int ixc = col_in ? ix : 0;
    const bool own = lane >= kLowerHaloX && lane < kWave - kLowerHaloX && col_in;
    const int r0 = rb * kLowerRows;
    const int cur = a.st[b].j & 1;
    const bool last = i == P.N - 1;
    const double *x = a.X[cur] + bi * n, *lam = a.LAM[cur] + bi * n;
    const double *xp = i == 0 ? a.x0 + (size_t)b * n : x - n;
    const double *ln = last ? lam : lam + n;   // not read at the last stage (value 0)
    const double *xr = a.xref + (size_t)b * a.xref_inst_stride + (size_t)i * a.xref_stage_stride;
    T *b1 = reinterpret_cast<T *>(a.b1) + bi * n, *b2 = reinterpret_cast<T *>(a.b2) + bi * n;
    T *invd = reinterpret_cast<T *>(a.invd) + bi * n, *cpk = reinterpret_cast<T *>(a.cpk) + bi * n;
    T *g2 = reinterpret_cast<T *>(a.g2) + bi * n;
    const double h = P.h, kp = P.k0 * P.k1, ax = P.idx2, ay = P.idy2;
    auto K = [&](double w) { return P.k0 * (1.0 + P.k1 * w); };
    // this lane's column sums of B u and gx column; this wave's gy rows in LDS
    // scb[bb] = sum_a gx[a][ix] u[bb lx + a] (the column factor of B u): lane
    // j holds u_j, the others read it with readlane
    double scb[kMaxLy];
    {
        const double ul = lane < P.m ? a.U[cur][bi * P.m + lane] : 0.0;
        const long long ub = __double_as_longlong(ul);
        const int ulo = (int)ub, uhi = (int)(ub >> 32);
        double gxv[kMaxLx];
#pragma unroll
        for (int aa = 0; aa < kMaxLx; ++aa) {
            const double gv = a.gx[(aa < P.lx ? aa : 0) * nsx + ixc];
            gxv[aa] = aa < P.lx && col_in ? gv : 0.0;
        }
#pragma unroll
        for (int bb = 0; bb < kMaxLy; ++bb) {
            double sum = 0.0;
#pragma unroll
            for (int aa = 0; aa < kMaxLx; ++aa) {
                const int j = bb < P.ly && aa < P.lx ? bb * P.lx + aa : 0;
                const long long w = ((long long)__builtin_amdgcn_readlane(uhi, j) << 32) |
                                    (long long)(unsigned)__builtin_amdgcn_readlane(ulo, j);
                sum += gxv[aa] * __longlong_as_double(w);
            }
            scb[bb] = bb < P.ly ? sum : 0.0;
        }
    }
    constexpr int NR = kLowerRows + 2;   // rows r0 - 1 .. r0 + kLowerRows
    constexpr int SLICE = 2 * kMaxLy * (kWave + 1);   // doubles per wave (>= NR kMaxLy)
    static_assert(NR * kMaxLy <= SLICE, "gy rows fit the wave's slice");
    __shared__ double slice[4][SLICE];
    double *gyl = slice[wv];   // [NR][kMaxLy], then [2][kMaxLy][65] for the partials
#pragma unroll
    for (int it = 0; it < (NR * kMaxLy + kWave - 1) / kWave; ++it) {
        const int e = lane + it * kWave;
        const int rr = e / kMaxLy, bb = e - rr * kMaxLy, row = r0 - 1 + rr;
        const bool ok = e < NR * kMaxLy && bb < P.ly && row >= 0 && row < nsy;
        const double v = a.gy[ok ? bb * nsy + row : 0];
        if (e < NR * kMaxLy) gyl[e] = ok ? v : 0.0;
    }
    constexpr int PFR = 2;
    static_assert(NR % PFR == 0, "whole groups of rows");
    double qx[PFR], ql[PFR], qp[PFR], qn[PFR], qr[PFR];
    auto load_row = [&](int k, double &vx, double &vl, double &vp, double &vn, double &vr) {
        const int pc = (k >= 0 && k < nsy ? k : 0) * nsx + ixc;
        vx = x[pc]; vl = lam[pc]; vp = xp[pc]; vn = ln[pc]; vr = xr[pc];
    };
#pragma unroll
    for (int t = 0; t < PFR; ++t) load_row(r0 - 1 + t, qx[t], ql[t], qp[t], qn[t], qr[t]);
    double x_2 = 0, x_1 = 0, x_0 = 0, g_2 = 0, g_1 = 0, g_0 = 0;
    double l_1 = 0, l_0 = 0, p_1 = 0, p_0 = 0, n_1 = 0, n_0 = 0, r_1 = 0, r_0 = 0;
    unsigned long long mx = 0, ml = 0;
    double cl[kMaxLy];
#pragma unroll
    for (int bb = 0; bb < kMaxLy; ++bb) cl[bb] = 0.0;
#pragma unroll 1
    for (int g0 = 0; g0 < NR; g0 += PFR)
#pragma unroll
    for (int st = 0; st < PFR; ++st) {
        const int kk = g0 + st, k = r0 - 1 + kk;
        x_2 = x_1; x_1 = x_0; g_2 = g_1; g_1 = g_0;
        l_1 = l_0; p_1 = p_0; n_1 = n_0; r_1 = r_0;
        const bool in = col_in && k >= 0 && k < nsy;
        const double vx = qx[st], vl = ql[st], vp = qp[st], vn = qn[st], vr = qr[st];
        load_row(k + PFR, qx[st], ql[st], qp[st], qn[st], qr[st]);
        x_0 = in ? vx : 0.0;
        l_0 = in ? vl : 0.0;
        p_0 = vp; n_0 = last ? 0.0 : vn; r_0 = vr;
        g_0 = K(x_0) * l_0;
        if (kk >= 2) {   // row r = k - 1 of the block
            const int r = k - 1;
            const double Lx = ax * (wshr(x_1) + wshl(x_1)) + ay * (x_2 + x_0) - P.c0 * x_1;
            const double Lg = ax * (wshr(g_1) + wshl(g_1)) + ay * (g_2 + g_0) - P.c0 * g_1;
            double bu = 0.0;
#pragma unroll
            for (int bb = 0; bb < kMaxLy; ++bb) bu += gyl[(kk - 1) * kMaxLy + bb] * scb[bb];
            const double kl = n_1 - l_1 + h * (P.q * (x_1 - r_1) + Lg + kp * Lx * l_1);
            const double kx = p_1 - x_1 + h * (K(x_1) * Lx + bu);
            const bool ok = own && r < nsy;
            const unsigned long long ax_ = sabits(kx), al_ = sabits(kl);
            mx = ok && ax_ > mx ? ax_ : mx;
            ml = ok && al_ > ml ? al_ : ml;
            const double lv = ok ? l_1 : 0.0;
#pragma unroll
            for (int bb = 0; bb < kMaxLy; ++bb) cl[bb] += gyl[(kk - 1) * kMaxLy + bb] * lv;
            if (ok) {
                const int p = r * nsx + ix;
                b1[p] = T(kx);
                b2[p] = T(kl);
                const double d = -1.0 - h * K(x_1) * P.c0 + h * kp * Lx;
                invd[p] = st_recip<T>(d);
                cpk[p] = T(h * K(x_1));
                g2[p] = T(kp * l_1);
            }
        }
    }
    // unit partials: norms (wave maxima) and B^T lambda over the owned lanes
    const long long upart = (bi * a.nrb + rb) * a.nstrip + sp;
    mx = wave_umax(mx);
    ml = wave_umax(ml);
    if (lane == 0) {
        a.unorm[2 * upart] = mx;
        a.unorm[2 * upart + 1] = ml;
    }
    double (*cs)[kWave + 1] = reinterpret_cast<double (*)[kWave + 1]>(gyl);
    double (*gs)[kWave + 1] = cs + kMaxLy;
#pragma unroll
    for (int q = 0; q < kMaxLy; ++q) {
        cs[q][lane] = own ? cl[q] : 0.0;
        const double gv = a.gx[(q < P.lx ? q : 0) * nsx + ixc];
        gs[q][lane] = q < P.lx && col_in ? gv : 0.0;
    }
    if (lane < P.m) {
        const int bb = lane / P.lx, aa = lane - bb * P.lx;
        double v = 0.0;
        for (int l = 0; l < kWave; ++l) v += cs[bb][l] * gs[aa][l];
        a.part[upart * kMaxM + lane] = v;
    }
}

// (B^T y)_{bb*lx+a} of stage bi from its rows' partials sum_ix gx[a][ix] y,
// for all j < m: a 256-thread workgroup splits the rows in four quarters
// (threads j, j + 64, ...) and sums the quarters through LDS; the result is
// valid in threads t < m.
__device__ __forceinline__ double bt_from_rows(const StreamArgs &a, size_t bi, double *sh)
{
    const int t = threadIdx.x, j = t & (kWave - 1), qtr = t / kWave, nq = (int)(blockDim.x / kWave);
    double s = 0.0;
    if (j < a.P.m) {
        const int bb = j / a.P.lx, aa = j % a.P.lx;
        for (int iy = qtr; iy < a.P.nsy; iy += nq)
            s += a.gy[bb * a.P.nsy + iy] * a.rowt[(bi * a.P.nsy + iy) * kMaxLx + aa];
    }
    sh[t] = s;
    __syncthreads();
    double tot = 0.0;
    if (t < kWave)
        for (int q = 0; q < nq; ++q) tot += sh[q * kWave + t];
    return tot;
}

// K^u, the stage's norms and v3 = 0 from the residual pass's unit partials.
// One workgroup (256 threads) per stage.
template <int PREC>
__global__ void __launch_bounds__(256) k_st_stage(const StreamArgs a)
{
    __shared__ unsigned long long shn[2 * kMaxWaves];
    const int bi = blockIdx.x;
    if (bi >= a.count * a.P.N) return;
    const int b = bi / a.P.N;
    if (!evaluating<PREC>(a, b)) return;
    const DevProblem &P = a.P;
    const int m = P.m, units = a.nrb * a.nstrip;
    const int cur = a.st[b].j & 1;
    unsigned long long mu = 0, mx = 0, ml = 0;
    if (threadIdx.x < m) {
        const int j = threadIdx.x;
        const double *pp = a.part + (size_t)bi * units * kMaxM + j;
        double bt = 0.0;
#pragma unroll 8
        for (int u = 0; u < units; ++u) bt += pp[(size_t)u * kMaxM];
        const double u = a.U[cur][(size_t)bi * m + j];
        double bg = 0.0;   // gradient of the input box's barrier (eq. nlp_relaxed)
        if (P.tau > 0.0) bg = -P.tau / (u - P.ulo) + P.tau / (P.uhi - u);
        const double ku = P.h * (P.r * u + bg + bt);
        a.kun[(size_t)bi * m + j] = ku;
        a.v3[(size_t)bi * m + j] = 0.0;
        mu = sabits(ku);
    }
    for (int u = threadIdx.x; u < units; u += blockDim.x) {
        mx = sumax(mx, a.unorm[2 * ((size_t)bi * units + u)]);
        ml = sumax(ml, a.unorm[2 * ((size_t)bi * units + u) + 1]);
    }
    mx = wave_umax(mx);
    ml = wave_umax(ml);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) { shn[2 * w] = mx; shn[2 * w + 1] = ml; }
    mu = wave_umax(mu);   // the inputs live in wave 0
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < (int)(blockDim.x / kWave); ++q) {
            mx = sumax(mx, shn[2 * q]);
            ml = sumax(ml, shn[2 * q + 1]);
        }
        const double dx = sbits2d(mx), dl = sbits2d(ml), du = sbits2d(mu);
        double rp = dx > du ? dx : du;
        rp = rp > dl ? rp : dl;
        double rs = dx, su = du / (P.h * P.r), sl = dl / P.h;
        rs = rs > su ? rs : su;
        rs = rs > sl ? rs : sl;
        const bool bad = mx >= 0x7FF0000000000000ull || ml >= 0x7FF0000000000000ull ||
                         mu >= 0x7FF0000000000000ull;
        if (bad) { rs = __longlong_as_double(0x7FF8000000000000ll); rp = rs; }
        a.rst[bi] = sabits(rs);
        a.pst[bi] = sabits(rp);
    }
}

// Per-instance decision of the graph of precision PREC (one thread per
// instance): FP32 mode passing the test -> REDO (left for the FP64 graph);
// REDO -> one FP64 step from S^j; FP64 mode passing -> finished.
template <int PREC>
__global__ void k_st_decide(const StreamArgs a)
{
    // one wave per instance: the lanes take the stage maxima, lane 0 decides
    const int b = blockIdx.x, lane = threadIdx.x;
    if (b >= a.count) return;
    if (!evaluating<PREC>(a, b)) {
        if (lane == 0) a.work[b] = 0;
        return;
    }
    unsigned long long ms = 0, mp = 0;
    for (int i = lane; i < a.P.N; i += kWave) {
        ms = sumax(ms, a.rst[(size_t)b * a.P.N + i]);
        mp = sumax(mp, a.pst[(size_t)b * a.P.N + i]);
    }
    ms = wave_umax(ms);
    mp = wave_umax(mp);
    if (lane != 0) return;
    InstState s = a.st[b];
    const double rs = sbits2d(ms), rp = sbits2d(mp);
    const double rt = a.res_paper ? rp : rs;   // the norm the test is on
    const bool was32 = s.mode == kModeFp32;
    int fin = -1, work = 0;
    if (!(rt <= 1.7976931348623157e308)) {
        fin = kStatusNonfinite;
    } else if (rt <= a.tol) {
        if (s.mode == kModeFp32) {
            s.mode = kModeFp64Redo;
        } else if (s.mode == kModeFp64Redo) {
            s.mode = kModeFp64;
            work = 2;   // the FP64 correction step from the FP32-sweep iterate
        } else {
            fin = kStatusOk;
        }
    } else if (s.j >= a.max_iter) {
        fin = kStatusNoconv;
    } else {
        work = s.mode == kModeFp64Redo ? 2 : 1;
        if (s.mode == kModeFp64Redo) s.mode = kModeFp64;
    }
    if (was32 && (s.mode != kModeFp32 || fin >= 0)) atomicSub(a.ctr + 3, 1);
    if (work) {
        ++s.e;
        if (PREC == kModeFp32) ++s.f32;
    }
    if (fin >= 0) {
        s.status = fin;
        a.iters[b] = s.j;
        a.rfin[2 * b] = rs;
        a.rfin[2 * b + 1] = rp;
        atomicAdd(a.ctr + 2, 1);
    }
    a.st[b] = s;
    a.work[b] = work;
}

// F_x solve (point-Jacobi from zero) of c = sgn (b1 - h B v3) (sgn = -1 in
// the Schur iterations, where c = h B v3 - b1; +1 in the final block).
// pass 0: c and the first sweep's values y1 = c / d of the block and halo
// rows are staged in LDS and the second sweep y = (c - cpk N(y1)) / d is
// written to y5 (one sweep: y1 itself); pass s >= 1: sweep s + 2 from y5 /
// ytmp (ping-pong by parity) staged in LDS.
template <typename T>
__global__ void __launch_bounds__(256) k_st_jf(const StreamArgs a, int sgn, int use_v3, int pass)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const Block u = row_block(a);
    if (!u.ok || !a.work[u.b]) return;
    const DevProblem &P = a.P;
    const int nsx = P.nsx, n = nsx * P.nsy;
    const size_t bi = (size_t)u.b * P.N + u.i;
    const T *b1 = reinterpret_cast<const T *>(a.b1) + bi * n;
    const T *invd = reinterpret_cast<const T *>(a.invd) + bi * n;
    const T *cpk = reinterpret_cast<const T *>(a.cpk) + bi * n;
    T *y5 = reinterpret_cast<T *>(a.y5) + bi * n, *yt = reinterpret_cast<T *>(a.ytmp) + bi * n;
    const T h = T(P.h), ax = T(P.idx2), ay = T(P.idy2);
    auto crow = [&](int iy, int ix, const BCol &cv) -> T {
        const T bv = use_v3 ? T(bsep_row(a, cv, iy)) : T(0);
        const T v = b1[iy * nsx + ix] - h * bv;
        return sgn > 0 ? v : -v;
    };
    auto rhs = [&](int iy, int ix) -> T {
        return crow(iy, ix, use_v3 ? bsep_col(a, bi, ix) : BCol{});
    };
    T *ys = reinterpret_cast<T *>(lds_raw);
    const int lane = threadIdx.x & (kWave - 1);
    if (pass == 0) {
        if (a.n_sw < 2) {
            own_rows(P, u.iy0, [&](int rr, int iy) {
                for (int ix = lane; ix < nsx; ix += kWave) y5[iy * nsx + ix] = rhs(iy, ix) * invd[iy * nsx + ix];
            });
            return;
        }
        T *cs = ys + (kRows + 2) * nsx;   // c of the block and halo rows
        for_staged(P, u.iy0, [&](int ix) { return use_v3 ? bsep_col(a, bi, ix) : BCol{}; },
                   [&](int e, int iy, int ix, bool in, const BCol &cv) {
                       const T cv_ = in ? crow(iy, ix, cv) : T(0);
                       cs[e] = cv_;
                       ys[e] = in ? cv_ * invd[iy * nsx + ix] : T(0);
                   });
        __syncthreads();
        own_rows(P, u.iy0, [&](int rr, int iy) {
            for (int ix = lane; ix < nsx; ix += kWave) {
                const int p = iy * nsx + ix;
                y5[p] = (cs[(rr + 1) * nsx + ix] - cpk[p] * lds_nb(ys, nsx, rr, ix, ax, ay)) * invd[p];
            }
        });
    } else {
        const T *yin = (pass & 1) ? y5 : yt;
        T *yout = (pass & 1) ? yt : y5;
        stage_rows(ys, P, u.iy0, [&](int iy, int ix) { return yin[iy * nsx + ix]; });
        own_rows(P, u.iy0, [&](int rr, int iy) {
            for (int ix = lane; ix < nsx; ix += kWave) {
                const int p = iy * nsx + ix;
                yout[p] = (rhs(iy, ix) - cpk[p] * lds_nb(ys, nsx, rr, ix, ax, ay)) * invd[p];
            }
        });
    }
}

// c' = sgn b2 - A_xx y5 (sgn = -1 in the Schur iterations: c' = -b2 - A_xx y5),
// A_xx y = h ((q - 2 c0 g2) y + g2 N(y) + N(g2 y)); y and g2 y of the block
// and halo rows staged in LDS. y5 is the F_x solve's result (in ytmp when its
// last pass was odd).
template <typename T>
__global__ void __launch_bounds__(256) k_st_axx(const StreamArgs a, int sgn, int y_in_tmp)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const Block u = row_block(a);
    if (!u.ok || !a.work[u.b]) return;
    const DevProblem &P = a.P;
    const int nsx = P.nsx, n = nsx * P.nsy;
    const size_t bi = (size_t)u.b * P.N + u.i;
    const T *y = reinterpret_cast<const T *>(y_in_tmp ? a.ytmp : a.y5) + bi * n;
    const T *g2 = reinterpret_cast<const T *>(a.g2) + bi * n;
    const T *b2 = reinterpret_cast<const T *>(a.b2) + bi * n;
    T *cp = reinterpret_cast<T *>(a.cp) + bi * n;
    const T ax = T(P.idx2), ay = T(P.idy2), h = T(P.h), q = T(P.q), c0 = T(P.c0);
    T *ys = reinterpret_cast<T *>(lds_raw);
    T *zs = ys + (kRows + 2) * nsx;
    for_staged(P, u.iy0, no_col, [&](int e, int iy, int ix, bool in, NoCol) {
        const int p = iy * nsx + ix;
        const T yv = in ? y[p] : T(0);
        ys[e] = yv;
        zs[e] = in ? g2[p] * yv : T(0);
    });
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    own_rows(P, u.iy0, [&](int rr, int iy) {
        for (int ix = lane; ix < nsx; ix += kWave) {
            const int p = iy * nsx + ix, e = (rr + 1) * nsx + ix;
            const T n1 = lds_nb(ys, nsx, rr, ix, ax, ay), n2 = lds_nb(zs, nsx, rr, ix, ax, ay);
            const T Ay = h * ((q - T(2) * c0 * g2[p]) * ys[e] + g2[p] * n1 + n2);
            cp[p] = (sgn > 0 ? b2[p] : -b2[p]) - Ay;
        }
    });
}

// F_x^T solve of c' into y4 (pass as in k_st_jf, ping-pong with y4tmp; the
// staged values are cpk times the previous sweep's); on the last pass
// optionally the row partials of B^T y4, and in the final block the update of
// x, lambda and u into the other iterate buffer.
template <typename T>
__global__ void __launch_bounds__(256) k_st_jft(const StreamArgs a, int pass, int last_pass,
                                                int partials, int update, int y5_in_tmp)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const Block u = row_block(a);
    if (!u.ok || !a.work[u.b]) return;
    const DevProblem &P = a.P;
    const int nsx = P.nsx, n = nsx * P.nsy;
    const size_t bi = (size_t)u.b * P.N + u.i;
    const T *invd = reinterpret_cast<const T *>(a.invd) + bi * n;
    const T *cpk = reinterpret_cast<const T *>(a.cpk) + bi * n;
    const T *cp = reinterpret_cast<const T *>(a.cp) + bi * n;
    T *y4 = reinterpret_cast<T *>(a.y4) + bi * n, *yt = reinterpret_cast<T *>(a.y4tmp) + bi * n;
    const T ax = T(P.idx2), ay = T(P.idy2);
    T *zs = reinterpret_cast<T *>(lds_raw);
    const int lane = threadIdx.x & (kWave - 1);
    T *res = y4;
    if (pass == 0 && a.n_sw < 2) {
        own_rows(P, u.iy0, [&](int rr, int iy) {
            for (int ix = lane; ix < nsx; ix += kWave) y4[iy * nsx + ix] = cp[iy * nsx + ix] * invd[iy * nsx + ix];
        });
    } else {
        const T *yin = pass == 0 ? nullptr : ((pass & 1) ? y4 : yt);
        res = pass == 0 ? y4 : ((pass & 1) ? yt : y4);
        stage_rows(zs, P, u.iy0, [&](int iy, int ix) {
            const int p = iy * nsx + ix;
            return cpk[p] * (pass == 0 ? cp[p] * invd[p] : yin[p]);
        });
        own_rows(P, u.iy0, [&](int rr, int iy) {
            for (int ix = lane; ix < nsx; ix += kWave) {
                const int p = iy * nsx + ix;
                res[p] = (cp[p] - lds_nb(zs, nsx, rr, ix, ax, ay)) * invd[p];
            }
        });
    }
    if (!last_pass) return;
    const int cur = a.st[u.b].j & 1, nxt = cur ^ 1;
    const T *y5 = reinterpret_cast<const T *>(y5_in_tmp ? a.ytmp : a.y5) + bi * n;
    own_rows(P, u.iy0, [&](int rr, int iy) {
        // this wave's own results of row iy are read back (same lanes)
        if (partials) {
            double tl[kMaxLx];
            for (int q = 0; q < P.lx; ++q) tl[q] = 0.0;
            for (int ix = lane; ix < nsx; ix += kWave) {
                const double yv = double(res[iy * nsx + ix]);
                for (int q = 0; q < P.lx; ++q) tl[q] += a.gx[q * nsx + ix] * yv;
            }
            for (int q = 0; q < P.lx; ++q) tl[q] = wave_sum(tl[q]);
            if (lane == 0) {
                const size_t ru = bi * P.nsy + iy;
                for (int q = 0; q < P.lx; ++q) a.rowt[ru * kMaxLx + q] = tl[q];
            }
        }
        if (update) {
            const double *x = a.X[cur] + bi * n, *lam = a.LAM[cur] + bi * n;
            double *xn = a.X[nxt] + bi * n, *ln = a.LAM[nxt] + bi * n;
            for (int ix = lane; ix < nsx; ix += kWave) {
                const int p = iy * nsx + ix;
                xn[p] = x[p] - double(y5[p]);
                ln[p] = lam[p] - double(res[p]);
            }
        }
    });
    if (update && u.iy0 == 0) {
        const double *uc = a.U[cur] + bi * P.m;
        double *un = a.U[nxt] + bi * P.m;
        const int b = (int)(bi / P.N);
        for (int j = threadIdx.x; j < P.m; j += blockDim.x) {
            un[j] = uc[j] - a.v3[bi * P.m + j];
            if (a.work[b] == 2 && a.du) {   // size of the FP64 correction step
                atomicMax(a.du + 2 * b, sabits(a.v3[bi * P.m + j]));
                atomicMax(a.du + 2 * b + 1, sabits(un[j]));
            }
        }
    }
}

// A_uu of input j of stage bi: h r + gamma, plus h times the Hessian of the
// input box's barrier at the stage's current input.
__device__ __forceinline__ double stream_auu(const StreamArgs &a, long long bi, int j)
{
    double au = a.P.h * a.P.r + a.P.gamma;
    if (a.P.tau > 0.0) {
        const int b = (int)(bi / a.P.N);
        const double u = a.U[a.st[b].j & 1][(size_t)bi * a.P.m + j];
        const double lo = u - a.P.ulo, hi = a.P.uhi - u;
        au += a.P.h * (a.P.tau / (lo * lo) + a.P.tau / (hi * hi));
    }
    return au;
}

// v3 = (K^u + h B^T y4) / A_uu per stage (T arithmetic as in the fused
// kernel). One workgroup (256 threads) per stage.
template <typename T>
__global__ void __launch_bounds__(256) k_st_v3(const StreamArgs a)
{
    __shared__ double sh[256];
    const int bi = blockIdx.x;
    if (bi >= a.count * a.P.N) return;
    const int b = bi / a.P.N;
    if (!a.work[b]) return;
    const T h = T(a.P.h);
    const double btd = bt_from_rows(a, bi, sh);
    if (threadIdx.x < a.P.m) {
        const int j = threadIdx.x;
        const T bt = T(btd);
        const T auu = T(stream_auu(a, bi, j));
        a.v3[(size_t)bi * a.P.m + j] = double((T(a.kun[(size_t)bi * a.P.m + j]) + h * bt) / auu);
    }
}

// Fused Schur step (fin = 0, sgn = -1) or final block (fin = 1, sgn = +1) of
// the lower layer for two point-Jacobi sweeps per solve, in one pass:
//   c  = sgn (b1 - h B v3),  y1 = c / d,  y5 = (c - cpk N(y1)) / d       (F_x solve)
//   c' = sgn b2 - A_xx y5,   z1 = cpk c' / d,  y4 = (c' - N(z1)) / d      (F_x^T solve)
// then the partial sums of B^T y4 (Schur step) or the update
// S^{k+1} = S^k - (y5, v3, y4) (final block). One wave per unit of
// kLowerRows rows and a strip of 64 columns whose 56 inner lanes own their
// column: horizontal neighbours come from the adjacent lanes (DPP wave
// shifts), vertical ones from the rows the lane has already visited, so the
// pass needs no LDS and no barrier. Each lane walks its column from three
// rows above the block to three rows below; every quantity trails the row
// being loaded by the rows its stencils need (y5 by 1, c' and z1 by 2, y4 by
// 3). Outside the grid d^-1 = 0 makes every value zero, which is the
// Dirichlet condition of the stencils. The halo lanes' values are wrong near
// the strip ends, and only the inner lanes are used.
// which < 0: v3 is read from a.v3 (zero after the stage kernel); which = 0 / 1:
// each wave forms v3 = (K^u + h B^T y4) / A_uu of its stage from the previous
// Schur step's unit partials in part / part2 (summed in unit order, T
// arithmetic as in the fused stage kernel), and a Schur step writes its own
// partials to the other buffer.
template <typename T, bool FIN>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 3 : 2) k_st_lower(const StreamArgs a,
                                                                                      int which)
{
    constexpr bool fin = FIN;
    const int lane = threadIdx.x & (kWave - 1);
    const long long g = (long long)(blockIdx.x & 7) * a.lper_xcd + (blockIdx.x >> 3);
    const long long unit = g * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (unit >= a.lunits) return;
    const int sp = (int)(unit % a.nstrip);
    const long long t1 = unit / a.nstrip;
    const int rb = (int)(t1 % a.nrb);
    const long long bi = t1 / a.nrb;
    const int b = (int)(bi / a.P.N);
    if (!a.work[b]) return;
    const DevProblem &P = a.P;
    const int nsx = P.nsx, nsy = P.nsy, n = nsx * nsy, m = P.m;
    const int ix = sp * kLowerCols - kLowerHaloX + lane;
    const bool col_in = ix >= 0 && ix < nsx;
    const bool own = lane >= kLowerHaloX && lane < kWave - kLowerHaloX && col_in;
    const int r0 = rb * kLowerRows;
    const T sgn = fin ? T(1) : T(-1);
    const T h = T(P.h), ax = T(P.idx2), ay = T(P.idy2), qw = T(P.q), c0 = T(P.c0);
    const T *b1 = reinterpret_cast<const T *>(a.b1) + bi * n;
    const T *b2 = reinterpret_cast<const T *>(a.b2) + bi * n;
    const T *invd = reinterpret_cast<const T *>(a.invd) + bi * n;
    const T *cpk = reinterpret_cast<const T *>(a.cpk) + bi * n;
    const T *g2 = reinterpret_cast<const T *>(a.g2) + bi * n;
    const int ixc = col_in ? ix : 0;   // in-range column for the factor tables
    // column factor of B v3: scol[bb] = sum_a gx[a][ix] v3[bb lx + a] (v3 is
    // exactly zero in the first Schur step, so c = sgn b1 there)
    // this lane's gx column (zero past lx and outside the grid); every load
    // below is independent and unrolled, so they are in flight together
    T gxv[kMaxLx];
#pragma unroll
    for (int aa = 0; aa < kMaxLx; ++aa) {
        const double g = a.gx[(aa < P.lx ? aa : 0) * nsx + ixc];
        gxv[aa] = aa < P.lx && col_in ? T(g) : T(0);
    }
    // v3 (m <= 64 values): lane j loads v3[j], the others read it with readlane
    T scol[kMaxLy];
    double v3l = 0.0;
    if (which < 0) {
        v3l = lane < m ? a.v3[bi * m + lane] : 0.0;
    } else if (lane < m) {
        const int units = a.nrb * a.nstrip;
        const double *pp = (which ? a.part2 : a.part) + (size_t)bi * units * kMaxM + lane;
        double sum = 0.0;
#pragma unroll 8
        for (int u = 0; u < units; ++u) sum += pp[(size_t)u * kMaxM];
        const T hT = T(a.P.h);
        const T auu = T(stream_auu(a, bi, lane));
        v3l = double((T(a.kun[(size_t)bi * m + lane]) + hT * T(sum)) / auu);
    }
    {
        const long long vb = __double_as_longlong(v3l);
        const int vlo = (int)vb, vhi = (int)(vb >> 32);
#pragma unroll
        for (int bb = 0; bb < kMaxLy; ++bb) {
            double s = 0.0;
#pragma unroll
            for (int aa = 0; aa < kMaxLx; ++aa) {
                const int j = bb < P.ly && aa < P.lx ? bb * P.lx + aa : 0;
                const long long w = ((long long)__builtin_amdgcn_readlane(vhi, j) << 32) |
                                    (long long)(unsigned)__builtin_amdgcn_readlane(vlo, j);
                s += double(gxv[aa]) * __longlong_as_double(w);
            }
            scol[bb] = bb < P.ly ? T(s) : T(0);
        }
    }
    // this wave's rows of the gy factors, zero-padded to kMaxLy lattice rows
    // and outside the grid, in its own LDS slice (read back by the same wave)
    constexpr int NR = kLowerRows + 2 * kLowerHalo;
    __shared__ T gys[4][NR][kMaxLy];
    T (*gyl)[kMaxLy] = gys[threadIdx.x / kWave];
#pragma unroll
    for (int it = 0; it < (NR * kMaxLy + kWave - 1) / kWave; ++it) {
        const int e = lane + it * kWave;
        const int rr = e / kMaxLy, bb = e - rr * kMaxLy, row = r0 - kLowerHalo + rr;
        const bool ok = e < NR * kMaxLy && bb < P.ly && row >= 0 && row < nsy;
        const double g = a.gy[ok ? bb * nsy + row : 0];
        if (e < NR * kMaxLy) gyl[rr][bb] = ok ? T(g) : T(0);
    }
    const int cur = a.st[b].j & 1, nxt = cur ^ 1;
    const double *xo = a.X[cur] + bi * n, *lo = a.LAM[cur] + bi * n;
    double *xn = a.X[nxt] + bi * n, *ln = a.LAM[nxt] + bi * n;
    T colsum[kMaxLy];
#pragma unroll
    for (int bb = 0; bb < kMaxLy; ++bb) colsum[bb] = T(0);
    // row windows (index: rows behind the row k loaded last)
    T c_1 = 0, c_0 = 0;
    T y1_2 = 0, y1_1 = 0, y1_0 = 0;
    T y5_3 = 0, y5_2 = 0, y5_1 = 0;
    T w_3 = 0, w_2 = 0, w_1 = 0;
    T cp_3 = 0, cp_2 = 0;
    T z_4 = 0, z_3 = 0, z_2 = 0;
    T d_3 = 0, d_2 = 0, d_1 = 0, d_0 = 0;
    T k_2 = 0, k_1 = 0, k_0 = 0;
    T g_2 = 0, g_1 = 0, g_0 = 0;
    T e_2 = 0, e_1 = 0, e_0 = 0;   // b2
    // the rows' coefficients are loaded PF rows ahead of their use into a
    // register ring; the loop runs in groups of PF rows with the group
    // unrolled, so step t of a group reads ring slot t and refills it with
    // the row PF steps ahead (no register moves of values still in flight)
    constexpr int PF = 6;
    static_assert((kLowerRows + 2 * kLowerHalo) % PF == 0, "whole groups of rows");
    T qd[PF], qk[PF], qg[PF], qe[PF], qb[PF];
    double qx[PF], ql[PF];   // final block: x and lambda of the row (for the update)
    // the final block reads x and lambda for the update anyway, so it forms the
    // coefficients from them (the residual pass's FP64 expressions, rounded to
    // T: the same values) instead of reading the stored ones
    auto load_row = [&](int k, int t) {
        const int kc = k >= 0 && k < nsy ? k : 0;   // in-range address, value masked later
        const int pc = kc * nsx + ixc;
        qe[t] = b2[pc]; qb[t] = b1[pc];
        if constexpr (FIN) {
            qx[t] = xo[pc];
            ql[t] = lo[pc];
        } else {
            qd[t] = invd[pc]; qk[t] = cpk[pc]; qg[t] = g2[pc];
        }
    };
#pragma unroll
    for (int t = 0; t < PF; ++t) load_row(r0 - kLowerHalo + t, t);
    double xw_1 = 0, xw_0 = 0, lw_3 = 0, lw_2 = 0, lw_1 = 0, lw_0 = 0;
    double xa = 0.0;   // final block: x of the row above the row being loaded (0 off the grid)
    if constexpr (FIN) {
        const int ka = r0 - kLowerHalo - 1;
        if (col_in && ka >= 0 && ka < nsy) xa = xo[ka * nsx + ix];
    }
    const double hd = P.h, kpd = P.k0 * P.k1;
#pragma unroll 1
    for (int g0 = 0; g0 < kLowerRows + 2 * kLowerHalo; g0 += PF)
#pragma unroll
    for (int st = 0; st < PF; ++st) {
        const int kk = g0 + st;
        const int k = r0 - kLowerHalo + kk;
        // shift the windows by one row
        c_1 = c_0; y1_2 = y1_1; y1_1 = y1_0;
        d_3 = d_2; d_2 = d_1; d_1 = d_0; k_2 = k_1; k_1 = k_0; g_2 = g_1; g_1 = g_0; e_2 = e_1; e_1 = e_0;
        // row k from ring slot st; row k + PF refills it
        const bool rin = k >= 0 && k < nsy, in = col_in && rin;
        T vd, vk, vg;
        const T ve = qe[st], vb = qb[st];
        if constexpr (FIN) {
            xw_1 = xw_0; lw_3 = lw_2; lw_2 = lw_1; lw_1 = lw_0;
            xw_0 = qx[st];
            lw_0 = ql[st];
            // coefficients of row k: L x from the rows above and below (the
            // ring's next slot holds row k + 1), as in the residual pass
            const double xk = in ? xw_0 : 0.0;
            const double xb = col_in && k + 1 >= 0 && k + 1 < nsy ? qx[(st + 1) % PF] : 0.0;
            const double Lx = P.idx2 * (wshr(xk) + wshl(xk)) + P.idy2 * (xa + xb) - P.c0 * xk;
            const double kk0 = P.k0 * (1.0 + P.k1 * xk);
            vd = st_recip<T>(-1.0 - hd * kk0 * P.c0 + hd * kpd * Lx);
            vk = T(hd * kk0);
            vg = T(kpd * (in ? lw_0 : 0.0));
            xa = xk;
        } else {
            vd = qd[st]; vk = qk[st]; vg = qg[st];
        }
        load_row(k + PF, st);
        T bu = 0;
#pragma unroll
        for (int bb = 0; bb < kMaxLy; ++bb) bu += gyl[kk][bb] * scol[bb];
        d_0 = in ? vd : T(0);
        k_0 = in ? vk : T(0);
        g_0 = in ? vg : T(0);
        e_0 = in ? ve : T(0);
        c_0 = in ? sgn * (vb - h * bu) : T(0);
        y1_0 = c_0 * d_0;
        // y5 and w at row k - 1
        if (kk >= 2) {
            y5_3 = y5_2; y5_2 = y5_1; w_3 = w_2; w_2 = w_1;
            const T nb = ax * (wshr(y1_1) + wshl(y1_1)) + ay * (y1_2 + y1_0);
            y5_1 = (c_1 - k_1 * nb) * d_1;
            w_1 = g_1 * y5_1;
            if constexpr (FIN) {
                const int r = k - 1;
                if (own && r >= r0 && r < r0 + kLowerRows && r < nsy) xn[r * nsx + ix] = xw_1 - double(y5_1);
            }
        }
        // c' and z1 at row k - 2
        if (kk >= 4) {
            cp_3 = cp_2; z_4 = z_3; z_3 = z_2;
            const T n1 = ax * (wshr(y5_2) + wshl(y5_2)) + ay * (y5_3 + y5_1);
            const T n2 = ax * (wshr(w_2) + wshl(w_2)) + ay * (w_3 + w_1);
            const T Ay = h * ((qw - T(2) * c0 * g_2) * y5_2 + g_2 * n1 + n2);
            cp_2 = sgn * e_2 - Ay;
            z_2 = k_2 * cp_2 * d_2;
        }
        // y4 at row k - 3
        if (kk >= 6) {
            const T nb = ax * (wshr(z_3) + wshl(z_3)) + ay * (z_4 + z_2);
            const T y4 = (cp_3 - nb) * d_3;
            const int r = k - 3;
            const bool upd = own && r < nsy;
            if constexpr (FIN) {
                if (upd) ln[r * nsx + ix] = lw_3 - double(y4);
            } else {
                const T y4o = upd ? y4 : T(0);
#pragma unroll
                for (int bb = 0; bb < kMaxLy; ++bb) colsum[bb] += gyl[kk - kLowerHalo][bb] * y4o;
            }
        }
    }
    const long long upart = (bi * a.nrb + rb) * a.nstrip + sp;
    if constexpr (FIN) {
        if (rb == 0 && sp == 0) {   // m <= 64: lane j holds v3_j
            const double *uc = a.U[cur] + bi * m;
            double *un = a.U[nxt] + bi * m;
            const int b = (int)(bi / a.P.N);
            if (lane < m) {
                const int j = lane;
                un[j] = uc[j] - v3l;
                a.v3[bi * m + j] = v3l;   // the step's input part (input-box rule)
                if (a.work[b] == 2 && a.du) {   // size of the FP64 correction step
                    atomicMax(a.du + 2 * b, sabits(v3l));
                    atomicMax(a.du + 2 * b + 1, sabits(un[j]));
                }
            }
        }
        return;
    }
    // partial (B^T y4)_{bb lx + a} of this unit: sum over the owned columns of
    // gx[a][ix] colsum[bb], reduced over the wave (m <= 64 values)
    // lane j < m sums gx[a][column] colsum[bb] over the strip's owned lanes,
    // read from this wave's LDS slice (rows padded to 65: no bank conflicts)
    __shared__ T strip[4][2][kMaxLy][kWave + 1];
    T (*cs)[kWave + 1] = strip[threadIdx.x / kWave][0];
    T (*gs)[kWave + 1] = strip[threadIdx.x / kWave][1];
#pragma unroll
    for (int q = 0; q < kMaxLy; ++q) {
        cs[q][lane] = own ? colsum[q] : T(0);
        gs[q][lane] = gxv[q];
    }
    if (lane < m) {
        const int bb = lane / P.lx, aa = lane - bb * P.lx;
        T v = 0;
        for (int l = 0; l < kWave; ++l) v += cs[bb][l] * gs[aa][l];
        (which == 0 ? a.part2 : a.part)[upart * kMaxM + lane] = double(v);
    }
}

// The residual pass fused with the first Schur step (two sweeps per solve,
// at least one Schur step). In the first step v3 = 0, so its right-hand side
// c = -b1 needs no reduction over the stage, and the step can trail the KKT
// rows in the same march: each lane walks its column from four rows above the
// block to four below; the KKT rows and coefficients (FP64, rounded to T as
// the stored ones) trail the loaded row by one, and the Schur step trails
// them as the lower pass trails its loaded row (y5 by 1, c' and z1 by 2, y4
// by 3). Four halo columns: each of the four stencils on the way to y4
// spoils one more column at the strip ends. Writes the lower layer's
// right-hand sides and coefficients for the later passes (block rows, owned
// columns), the unit partials of the norms and of B^T lambda (part) and of
// B^T y4 (part2). The arithmetic is that of k_st_res followed by k_st_lower
// with v3 = 0, so the iterates do not change.
template <typename T>
__global__ void __launch_bounds__(256, 2) k_st_res1(const StreamArgs a)
{
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const long long gu = (long long)(blockIdx.x & 7) * a.lper_xcd + (blockIdx.x >> 3);
    const long long unit = gu * (blockDim.x / kWave) + wv;
    if (unit >= a.lunits) return;
    const int sp = (int)(unit % a.nstrip);
    const long long t1 = unit / a.nstrip;
    const int rb = (int)(t1 % a.nrb);
    const long long bi = t1 / a.nrb;
    const int b = (int)(bi / a.P.N), i = (int)(bi % a.P.N);
    constexpr int PREC = std::is_same<T, float>::value ? kModeFp32 : kModeFp64;
    if (!evaluating<PREC>(a, b)) return;
    const DevProblem &P = a.P;
    const int nsx = P.nsx, nsy = P.nsy, n = nsx * nsy;
    const int ix = sp * kLowerCols - kLowerHaloX + lane;
    const bool col_in = ix >= 0 && ix < nsx;
    const int ixc = col_in ? ix : 0;
    const bool own = lane >= kLowerHaloX && lane < kWave - kLowerHaloX && col_in;
    const int r0 = rb * kLowerRows;
    const int cur = a.st[b].j & 1;
    const bool last = i == P.N - 1;
    const double *x = a.X[cur] + bi * n, *lam = a.LAM[cur] + bi * n;
    const double *xp = i == 0 ? a.x0 + (size_t)b * n : x - n;
    const double *ln = last ? lam : lam + n;   // not read at the last stage (value 0)
    const double *xr = a.xref + (size_t)b * a.xref_inst_stride + (size_t)i * a.xref_stage_stride;
    T *b1 = reinterpret_cast<T *>(a.b1) + bi * n, *b2 = reinterpret_cast<T *>(a.b2) + bi * n;
    T *invd = reinterpret_cast<T *>(a.invd) + bi * n, *cpk = reinterpret_cast<T *>(a.cpk) + bi * n;
    T *g2 = reinterpret_cast<T *>(a.g2) + bi * n;
    const double h = P.h, kp = P.k0 * P.k1, ax = P.idx2, ay = P.idy2;
    const T hT = T(P.h), axT = T(P.idx2), ayT = T(P.idy2), qT = T(P.q), c0T = T(P.c0);
    auto K = [&](double w) { return P.k0 * (1.0 + P.k1 * w); };
    // the column factor of B u for this lane (lane j holds u_j)
    double scb[kMaxLy];
    {
        const double ul = lane < P.m ? a.U[cur][bi * P.m + lane] : 0.0;
        const long long ub = __double_as_longlong(ul);
        const int ulo = (int)ub, uhi = (int)(ub >> 32);
        double gxv[kMaxLx];
#pragma unroll
        for (int aa = 0; aa < kMaxLx; ++aa) {
            const double gv = a.gx[(aa < P.lx ? aa : 0) * nsx + ixc];
            gxv[aa] = aa < P.lx && col_in ? gv : 0.0;
        }
#pragma unroll
        for (int bb = 0; bb < kMaxLy; ++bb) {
            double sum = 0.0;
#pragma unroll
            for (int aa = 0; aa < kMaxLx; ++aa) {
                const int j = bb < P.ly && aa < P.lx ? bb * P.lx + aa : 0;
                const long long w = ((long long)__builtin_amdgcn_readlane(uhi, j) << 32) |
                                    (long long)(unsigned)__builtin_amdgcn_readlane(ulo, j);
                sum += gxv[aa] * __longlong_as_double(w);
            }
            scb[bb] = bb < P.ly ? sum : 0.0;
        }
    }
    constexpr int HY = kLowerHalo + 1;             // rows above / below the block
    constexpr int NR = kLowerRows + 2 * HY;        // rows r0 - HY .. r0 + kLowerRows + HY - 1
    constexpr int SLICE = 2 * kMaxLy * (kWave + 1);   // doubles per wave (>= NR kMaxLy)
    static_assert(NR * kMaxLy <= SLICE, "gy rows fit the wave's slice");
    __shared__ double slice[4][SLICE];
    double *gyl = slice[wv];   // [NR][kMaxLy], then [2][kMaxLy][65] for the partials
#pragma unroll
    for (int it = 0; it < (NR * kMaxLy + kWave - 1) / kWave; ++it) {
        const int e = lane + it * kWave;
        const int rr = e / kMaxLy, bb = e - rr * kMaxLy, row = r0 - HY + rr;
        const bool ok = e < NR * kMaxLy && bb < P.ly && row >= 0 && row < nsy;
        const double v = a.gy[ok ? bb * nsy + row : 0];
        if (e < NR * kMaxLy) gyl[e] = ok ? v : 0.0;
    }
    constexpr int PFR = 2;
    static_assert(NR % PFR == 0, "whole groups of rows");
    double qx[PFR], ql[PFR], qp[PFR], qn[PFR], qr[PFR];
    auto load_row = [&](int k, double &vx, double &vl, double &vp, double &vn, double &vr) {
        const int pc = (k >= 0 && k < nsy ? k : 0) * nsx + ixc;
        vx = x[pc]; vl = lam[pc]; vp = xp[pc]; vn = ln[pc]; vr = xr[pc];
    };
#pragma unroll
    for (int t = 0; t < PFR; ++t) load_row(r0 - HY + t, qx[t], ql[t], qp[t], qn[t], qr[t]);
    // KKT windows (FP64)
    double x_2 = 0, x_1 = 0, x_0 = 0, g_2 = 0, g_1 = 0, g_0 = 0;
    double l_1 = 0, l_0 = 0, p_1 = 0, p_0 = 0, n_1 = 0, n_0 = 0, r_1 = 0, r_0 = 0;
    unsigned long long mx = 0, ml = 0;
    double cl[kMaxLy];
#pragma unroll
    for (int bb = 0; bb < kMaxLy; ++bb) cl[bb] = 0.0;
    // Schur-step windows (T), indexed by rows behind the newest KKT row
    T c_1 = 0, c_0 = 0;
    T y1_2 = 0, y1_1 = 0, y1_0 = 0;
    T y5_3 = 0, y5_2 = 0, y5_1 = 0;
    T w_3 = 0, w_2 = 0, w_1 = 0;
    T cp_3 = 0, cp_2 = 0;
    T z_4 = 0, z_3 = 0, z_2 = 0;
    T d_3 = 0, d_2 = 0, d_1 = 0, d_0 = 0;
    T k_2 = 0, k_1 = 0, k_0 = 0;
    T gg_2 = 0, gg_1 = 0, gg_0 = 0;
    T e_2 = 0, e_1 = 0, e_0 = 0;   // b2
    T colsum[kMaxLy];
#pragma unroll
    for (int bb = 0; bb < kMaxLy; ++bb) colsum[bb] = T(0);
#pragma unroll 1
    for (int g0 = 0; g0 < NR; g0 += PFR)
#pragma unroll
    for (int st = 0; st < PFR; ++st) {
        const int kk = g0 + st, k = r0 - HY + kk;
        x_2 = x_1; x_1 = x_0; g_2 = g_1; g_1 = g_0;
        l_1 = l_0; p_1 = p_0; n_1 = n_0; r_1 = r_0;
        const bool in = col_in && k >= 0 && k < nsy;
        const double vx = qx[st], vl = ql[st], vp = qp[st], vn = qn[st], vr = qr[st];
        load_row(k + PFR, qx[st], ql[st], qp[st], qn[st], qr[st]);
        x_0 = in ? vx : 0.0;
        l_0 = in ? vl : 0.0;
        p_0 = vp; n_0 = last ? 0.0 : vn; r_0 = vr;
        g_0 = K(x_0) * l_0;
        if (kk < 2) continue;
        // ---- KKT rows and coefficients of row r = k - 1
        const int r = k - 1;
        const bool rin = col_in && r >= 0 && r < nsy;
        const double Lx = ax * (wshr(x_1) + wshl(x_1)) + ay * (x_2 + x_0) - P.c0 * x_1;
        const double Lg = ax * (wshr(g_1) + wshl(g_1)) + ay * (g_2 + g_0) - P.c0 * g_1;
        double bu = 0.0;
#pragma unroll
        for (int bb = 0; bb < kMaxLy; ++bb) bu += gyl[(kk - 1) * kMaxLy + bb] * scb[bb];
        const double kl = n_1 - l_1 + h * (P.q * (x_1 - r_1) + Lg + kp * Lx * l_1);
        const double kx = p_1 - x_1 + h * (K(x_1) * Lx + bu);
        const double dd = -1.0 - h * K(x_1) * P.c0 + h * kp * Lx;
        const T tb1 = T(kx), tb2 = T(kl), tinvd = st_recip<T>(dd), tcpk = T(h * K(x_1));
        const T tg2 = T(kp * l_1);
        const bool blk = own && r >= r0 && r < r0 + kLowerRows && r < nsy;
        {
            const unsigned long long ax_ = sabits(kx), al_ = sabits(kl);
            mx = blk && ax_ > mx ? ax_ : mx;
            ml = blk && al_ > ml ? al_ : ml;
            const double lv = blk ? l_1 : 0.0;
#pragma unroll
            for (int bb = 0; bb < kMaxLy; ++bb) cl[bb] += gyl[(kk - 1) * kMaxLy + bb] * lv;
            if (blk) {
                const int pp = r * nsx + ix;
                b1[pp] = tb1;
                b2[pp] = tb2;
                invd[pp] = tinvd;
                cpk[pp] = tcpk;
                g2[pp] = tg2;
            }
        }
        // ---- first Schur step (v3 = 0): row r enters as the lower pass's loaded row
        const int kl2 = kk - 2;   // that pass's row counter (row r0 - kLowerHalo + kl2)
        c_1 = c_0; y1_2 = y1_1; y1_1 = y1_0;
        d_3 = d_2; d_2 = d_1; d_1 = d_0; k_2 = k_1; k_1 = k_0; gg_2 = gg_1; gg_1 = gg_0;
        e_2 = e_1; e_1 = e_0;
        d_0 = rin ? tinvd : T(0);
        k_0 = rin ? tcpk : T(0);
        gg_0 = rin ? tg2 : T(0);
        e_0 = rin ? tb2 : T(0);
        c_0 = rin ? T(-1) * (tb1 - hT * T(0)) : T(0);
        y1_0 = c_0 * d_0;
        if (kl2 >= 2) {   // y5 and w at row r - 1
            y5_3 = y5_2; y5_2 = y5_1; w_3 = w_2; w_2 = w_1;
            const T nb = axT * (wshr(y1_1) + wshl(y1_1)) + ayT * (y1_2 + y1_0);
            y5_1 = (c_1 - k_1 * nb) * d_1;
            w_1 = gg_1 * y5_1;
        }
        if (kl2 >= 4) {   // c' and z1 at row r - 2
            cp_3 = cp_2; z_4 = z_3; z_3 = z_2;
            const T n1 = axT * (wshr(y5_2) + wshl(y5_2)) + ayT * (y5_3 + y5_1);
            const T n2 = axT * (wshr(w_2) + wshl(w_2)) + ayT * (w_3 + w_1);
            const T Ay = hT * ((qT - T(2) * c0T * gg_2) * y5_2 + gg_2 * n1 + n2);
            cp_2 = T(-1) * e_2 - Ay;
            z_2 = k_2 * cp_2 * d_2;
        }
        if (kl2 >= 6) {   // y4 at row r - 3 (a block row)
            const T nb = axT * (wshr(z_3) + wshl(z_3)) + ayT * (z_4 + z_2);
            const T y4 = (cp_3 - nb) * d_3;
            const int ry = r - 3;
            const T y4o = own && ry < nsy ? y4 : T(0);
            const int gr = ry - (r0 - HY);   // gy table row
#pragma unroll
            for (int bb = 0; bb < kMaxLy; ++bb) colsum[bb] += T(gyl[gr * kMaxLy + bb]) * y4o;
        }
    }
    // unit partials: norms, B^T lambda (part) and B^T y4 (part2) over the owned lanes
    const long long upart = (bi * a.nrb + rb) * a.nstrip + sp;
    mx = wave_umax(mx);
    ml = wave_umax(ml);
    if (lane == 0) {
        a.unorm[2 * upart] = mx;
        a.unorm[2 * upart + 1] = ml;
    }
    double (*cs)[kWave + 1] = reinterpret_cast<double (*)[kWave + 1]>(gyl);
    double (*gs)[kWave + 1] = cs + kMaxLy;
#pragma unroll
    for (int q = 0; q < kMaxLy; ++q) {
        cs[q][lane] = own ? cl[q] : 0.0;
        const double gv = a.gx[(q < P.lx ? q : 0) * nsx + ixc];
        gs[q][lane] = q < P.lx && col_in ? gv : 0.0;
    }
    if (lane < P.m) {
        const int bb = lane / P.lx, aa = lane - bb * P.lx;
        double v = 0.0;
        for (int l = 0; l < kWave; ++l) v += cs[bb][l] * gs[aa][l];
        a.part[upart * kMaxM + lane] = v;
    }
    // B^T y4 in T, as the lower pass forms it
#pragma unroll
    for (int q = 0; q < kMaxLy; ++q) cs[q][lane] = own ? double(colsum[q]) : 0.0;
    if (lane < P.m) {
        const int bb = lane / P.lx, aa = lane - bb * P.lx;
        T v = 0;
        for (int l = 0; l < kWave; ++l) v += T(cs[bb][l]) * T(gs[aa][l]);
        a.part2[upart * kMaxM + lane] = double(v);
    }
}


// Input box, after the final block (the step S^{j+1} = S^j - ds written):
// each stage's fraction-to-the-boundary limit from its input step v3 (one
// wave per stage), then alpha = the instance's minimum scales the step where
// it is below 1 (eq. eq_alphamax; one workgroup per stage).
__global__ void k_st_box_lim(const StreamArgs a)
{
    const int bi = blockIdx.x, lane = threadIdx.x;
    if (bi >= a.count * a.P.N) return;
    const int b = bi / a.P.N;
    if (!a.work[b]) return;
    const int cur = a.st[b].j & 1;
    double l = 1.0;
    for (int j = lane; j < a.P.m; j += kWave) {
        const double u = a.U[cur][(size_t)bi * a.P.m + j], d = a.v3[(size_t)bi * a.P.m + j];
        double lj = 1.0;
        if (d > 0.0) lj = 0.995 * (u - a.P.ulo) / d;
        else if (d < 0.0) lj = 0.995 * (a.P.uhi - u) / (-d);
        l = fmin(l, fmax(lj, 0.0));
    }
    for (int o = 32; o >= 1; o >>= 1) l = fmin(l, __shfl_xor(l, o, kWave));
    if (lane == 0) a.apart[bi] = l;
}

__global__ void __launch_bounds__(256) k_st_box_apply(const StreamArgs a)
{
    __shared__ double red[256];
    const int bi = blockIdx.x;
    if (bi >= a.count * a.P.N) return;
    const int b = bi / a.P.N;
    if (!a.work[b]) return;
    double l = 1.0;
    for (int t = threadIdx.x; t < a.P.N; t += blockDim.x) l = fmin(l, a.apart[(size_t)b * a.P.N + t]);
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const double alpha = red[0];
    if (!(alpha < 1.0)) return;
    const int cur = a.st[b].j & 1, nxt = cur ^ 1;
    const size_t n = (size_t)a.P.nsx * a.P.nsy, so = (size_t)bi * n, uo = (size_t)bi * a.P.m;
    for (size_t p = threadIdx.x; p < n; p += blockDim.x) {
        const double xs = a.X[cur][so + p], ls = a.LAM[cur][so + p];
        a.X[nxt][so + p] = xs + alpha * (a.X[nxt][so + p] - xs);
        a.LAM[nxt][so + p] = ls + alpha * (a.LAM[nxt][so + p] - ls);
    }
    for (int j = threadIdx.x; j < a.P.m; j += blockDim.x) {
        const double us = a.U[cur][uo + j];
        a.U[nxt][uo + j] = us + alpha * (a.U[nxt][uo + j] - us);
    }
}

// j <- j + 1 for the instances that stepped (after every pass has used j).
__global__ void k_st_advance(const StreamArgs a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.count || !a.work[b]) return;
    a.st[b].j += 1;
}

StreamKernels stream_kernels(int prec)
{
    StreamKernels k{};
    k.advance = (const void *)&k_st_advance;
    k.box_lim = (const void *)&k_st_box_lim;
    k.box_apply = (const void *)&k_st_box_apply;
    if (prec == kModeFp32) {
        k.bsep = (const void *)&k_st_bsep<kModeFp32>;
        k.stage = (const void *)&k_st_stage<kModeFp32>;
        k.res = (const void *)&k_st_res<float>;
        k.decide = (const void *)&k_st_decide<kModeFp32>;
        k.jf = (const void *)&k_st_jf<float>;
        k.axx = (const void *)&k_st_axx<float>;
        k.jft = (const void *)&k_st_jft<float>;
        k.v3 = (const void *)&k_st_v3<float>;
        k.lower = (const void *)&k_st_lower<float, false>;
        k.lower_fin = (const void *)&k_st_lower<float, true>;
        k.res1 = (const void *)&k_st_res1<float>;
    } else {
        k.bsep = (const void *)&k_st_bsep<kModeFp64>;
        k.stage = (const void *)&k_st_stage<kModeFp64>;
        k.res = (const void *)&k_st_res<double>;
        k.decide = (const void *)&k_st_decide<kModeFp64>;
        k.jf = (const void *)&k_st_jf<double>;
        k.axx = (const void *)&k_st_axx<double>;
        k.jft = (const void *)&k_st_jft<double>;
        k.v3 = (const void *)&k_st_v3<double>;
        k.lower = (const void *)&k_st_lower<double, false>;
        k.lower_fin = (const void *)&k_st_lower<double, true>;
        k.res1 = (const void *)&k_st_res1<double>;
    }
    return k;
}

}  // namespace nmpc
