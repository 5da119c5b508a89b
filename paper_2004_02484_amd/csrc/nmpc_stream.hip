// nmpc_stream.hip -- streaming kernels of the Jacobi upper iteration for grids
// whose stage does not fit one workgroup (e.g. 256 x 256): every step of the
// stage algebra is a pass over all (instance, stage, grid row) units, one
// workgroup per row, with stencil neighbours read from the adjacent rows
// (L2-resident: each XCD receives a contiguous run of rows) and per-row
// partial reductions combined by small per-stage kernels.
//
// One upper iteration (eq. 1st_jacobi, alpha = 1), per instance and stage i:
//   K_res    KKT rows K^x, K^lambda (FP64), stage coefficients, row partials
//            of the norms and of B^T lambda
//   K_stage  K^u = h (r u + B^T lambda), the stage's norms, v3 = 0
//   decide   per-instance state machine (test, phases, max_iter)
//   Schur iterations (Sec. 5.2):  y5 = JacF(h B v3 - b1); c' = -b2 - A_xx y5;
//            y4 = JacFT(c'), row partials of B^T y4; v3 = (K^u + h B^T y4)/A_uu
//   final:   y5 = JacF(b1 - h B v3); y4 = JacFT(b2 - A_xx y5);
//            S^{k+1} = S^k - (y5, v3, y4)
// A point-Jacobi solve with n_sweep sweeps from zero is one pass for the
// first two sweeps (the first sweep's value c / d at a neighbour is formed on
// the fly) and one pass per further sweep.
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

// Row unit of a pass: XCD-aware order (each XCD a contiguous run of rows).
struct RowUnit {
    int b, i, iy;
    bool ok;
};

__device__ __forceinline__ RowUnit row_unit(const StreamArgs &a)
{
    RowUnit r{};
    const int bid = blockIdx.x;
    const long long unit = (long long)(bid & 7) * a.per_xcd + (bid >> 3);
    if (unit >= a.units) { r.ok = false; return r; }
    r.iy = (int)(unit % a.P.nsy);
    const long long bi = unit / a.P.nsy;
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

// Block-wide sum / max over 256 threads (4 waves) into thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < (int)(blockDim.x / kWave); ++q) s += sh[q];
    return s;
}

__device__ __forceinline__ unsigned long long block_max(unsigned long long v, unsigned long long *sh)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = sumax(v, __shfl_xor(v, m, kWave));
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) sh[w] = v;
    __syncthreads();
    unsigned long long s = 0;
    if (threadIdx.x == 0)
        for (int q = 0; q < (int)(blockDim.x / kWave); ++q) s = sumax(s, sh[q]);
    return s;
}

}  // namespace

// sc[b][i][bb][ix] = sum_a gx[a][ix] v[b][i][bb * lx + a]  (which = 0: U of
// the current iterate, for the instances this graph evaluates; 1: v3, for
// those it steps); (B v)_p = sum_bb gy[bb][iy] sc[bb][ix]. One workgroup per
// (instance, stage).
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

// KKT rows, coefficients and row partials of S^j (FP64 arithmetic; the
// right-hand sides and coefficients are stored in T for the lower layer).
template <typename T>
__global__ void __launch_bounds__(256) k_st_res(const StreamArgs a)
{
    __shared__ double sh[kMaxWaves];
    __shared__ unsigned long long shu[kMaxWaves];
    const RowUnit u = row_unit(a);
    if (!u.ok) return;
    const int PREC = std::is_same<T, float>::value ? kModeFp32 : kModeFp64;
    if (!evaluating<PREC>(a, u.b)) return;
    const DevProblem &P = a.P;
    const int n = P.nsx * P.nsy, nsx = P.nsx, nsy = P.nsy, iy = u.iy;
    const size_t bi = (size_t)u.b * P.N + u.i;
    const int cur = a.st[u.b].j & 1;
    const double *x = a.X[cur] + bi * n, *lam = a.LAM[cur] + bi * n;
    const double *xp = u.i == 0 ? a.x0 + (size_t)u.b * n : x - n;
    const double *ln = lam + n;
    const bool last = u.i == P.N - 1;
    const double *xr = a.xref + (size_t)u.b * a.xref_inst_stride + (size_t)u.i * a.xref_stage_stride;
    T *b1 = reinterpret_cast<T *>(a.b1) + bi * n, *b2 = reinterpret_cast<T *>(a.b2) + bi * n;
    T *invd = reinterpret_cast<T *>(a.invd) + bi * n, *cpk = reinterpret_cast<T *>(a.cpk) + bi * n;
    T *g2 = reinterpret_cast<T *>(a.g2) + bi * n;
    const double h = P.h, kp = P.k0 * P.k1;
    auto K = [&](double w) { return P.k0 * (1.0 + P.k1 * w); };
    unsigned long long mx = 0, ml = 0;
    double tl[kMaxLx];
    for (int q = 0; q < P.lx; ++q) tl[q] = 0.0;
    for (int ix = threadIdx.x; ix < nsx; ix += blockDim.x) {
        const int p = iy * nsx + ix;
        auto at = [&](const double *v, int dx, int dy) {
            const int jx = ix + dx, jy = iy + dy;
            return (jx < 0 || jx >= nsx || jy < 0 || jy >= nsy) ? 0.0 : v[jy * nsx + jx];
        };
        const double xc = x[p], lc = lam[p];
        const double Lx = P.idx2 * (at(x, -1, 0) + at(x, 1, 0)) + P.idy2 * (at(x, 0, -1) + at(x, 0, 1))
                          - P.c0 * xc;
        auto g = [&](int dx, int dy) {
            const int jx = ix + dx, jy = iy + dy;
            if (jx < 0 || jx >= nsx || jy < 0 || jy >= nsy) return 0.0;
            const int q = jy * nsx + jx;
            return K(x[q]) * lam[q];
        };
        const double gc = K(xc) * lc;
        const double Lg = P.idx2 * (g(-1, 0) + g(1, 0)) + P.idy2 * (g(0, -1) + g(0, 1)) - P.c0 * gc;
        const double kl = (last ? 0.0 : ln[p]) - lc + h * (P.q * (xc - xr[p]) + Lg + kp * Lx * lc);
        const double kx = xp[p] - xc + h * (K(xc) * Lx + bsep_at(a, bi, iy, ix));
        mx = sumax(mx, sabits(kx));
        ml = sumax(ml, sabits(kl));
        b1[p] = T(kx);
        b2[p] = T(kl);
        const double d = -1.0 - h * K(xc) * P.c0 + h * kp * Lx;
        invd[p] = T(1.0 / d);
        cpk[p] = T(h * K(xc));
        g2[p] = T(kp * lc);
        for (int q = 0; q < P.lx; ++q) tl[q] += a.gx[q * nsx + ix] * lc;
    }
    const size_t ru = bi * nsy + iy;
    const unsigned long long bx = block_max(mx, shu);
    if (threadIdx.x == 0) a.rown[2 * ru] = bx;
    const unsigned long long bl = block_max(ml, shu);
    if (threadIdx.x == 0) a.rown[2 * ru + 1] = bl;
    for (int q = 0; q < P.lx; ++q) {
        const double s = block_sum(tl[q], sh);
        if (threadIdx.x == 0) a.rowt[ru * kMaxLx + q] = s;
    }
}

// (B^T y)_{bb*lx+a} of stage bi from its rows' partials sum_ix gx[a][ix] y.
__device__ __forceinline__ double bt_from_rows(const StreamArgs &a, size_t bi, int j)
{
    const int bb = j / a.P.lx, aa = j % a.P.lx;
    double s = 0.0;
    for (int iy = 0; iy < a.P.nsy; ++iy)
        s += a.gy[bb * a.P.nsy + iy] * a.rowt[(bi * a.P.nsy + iy) * kMaxLx + aa];
    return s;
}

// K^u, the stage's norms and v3 = 0. One workgroup (64 threads) per stage.
template <int PREC>
__global__ void k_st_stage(const StreamArgs a)
{
    const int bi = blockIdx.x;
    if (bi >= a.count * a.P.N) return;
    const int b = bi / a.P.N;
    if (!evaluating<PREC>(a, b)) return;
    const DevProblem &P = a.P;
    const int m = P.m;
    const int cur = a.st[b].j & 1;
    unsigned long long mu = 0, mx = 0, ml = 0;
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        const double ku = P.h * (P.r * a.U[cur][(size_t)bi * m + j] + bt_from_rows(a, bi, j));
        a.kun[(size_t)bi * m + j] = ku;
        a.v3[(size_t)bi * m + j] = 0.0;
        mu = sumax(mu, sabits(ku));
    }
    for (int iy = threadIdx.x; iy < P.nsy; iy += blockDim.x) {
        mx = sumax(mx, a.rown[2 * ((size_t)bi * P.nsy + iy)]);
        ml = sumax(ml, a.rown[2 * ((size_t)bi * P.nsy + iy) + 1]);
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        mu = sumax(mu, __shfl_xor(mu, s, kWave));
        mx = sumax(mx, __shfl_xor(mx, s, kWave));
        ml = sumax(ml, __shfl_xor(ml, s, kWave));
    }
    if (threadIdx.x == 0) {
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
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.count) return;
    a.work[b] = 0;
    if (!evaluating<PREC>(a, b)) return;
    InstState s = a.st[b];
    unsigned long long ms = 0, mp = 0;
    for (int i = 0; i < a.P.N; ++i) {
        ms = sumax(ms, a.rst[(size_t)b * a.P.N + i]);
        mp = sumax(mp, a.pst[(size_t)b * a.P.N + i]);
    }
    const double rs = sbits2d(ms), rp = sbits2d(mp);
    const bool was32 = s.mode == kModeFp32;
    int fin = -1, work = 0;
    if (!(rs <= 1.7976931348623157e308)) {
        fin = kStatusNonfinite;
    } else if (rs <= a.tol) {
        if (s.mode == kModeFp32) {
            s.mode = kModeFp64Redo;
        } else if (s.mode == kModeFp64Redo) {
            s.mode = kModeFp64;
            work = 1;
        } else {
            fin = kStatusOk;
        }
    } else if (s.j >= a.max_iter) {
        fin = kStatusNoconv;
    } else {
        if (s.mode == kModeFp64Redo) s.mode = kModeFp64;
        work = 1;
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

// First pass of a point-Jacobi solve of F_x y = c (transposed: F_x^T y = c)
// from zero, with the right-hand side c formed per point by rhs():
//   one sweep:  y = c / d
//   two sweeps: y = (c - off) / d, off = sum of the neighbours' coupling to
//               their first-sweep values c_q / d_q
// F_x couples p to q with h k_p / dx^2 (row scaling by cpk_p); F_x^T with
// h k_q / dx^2 (the neighbour's cpk_q).
template <typename T, bool TRANS, typename RHS>
__device__ __forceinline__ void jacobi_first(const StreamArgs &a, const RowUnit &u, size_t bi,
                                             int nsw, const T *invd, const T *cpk, T *y, RHS rhs)
{
    const DevProblem &P = a.P;
    const int nsx = P.nsx, nsy = P.nsy, iy = u.iy;
    const T ax = T(P.idx2), ay = T(P.idy2);
    for (int ix = threadIdx.x; ix < nsx; ix += blockDim.x) {
        const int p = iy * nsx + ix;
        const T c = rhs(iy, ix);
        if (nsw < 2) { y[p] = c * invd[p]; continue; }
        auto y1 = [&](int dx, int dy) -> T {   // first-sweep value (times cpk for F^T)
            const int jx = ix + dx, jy = iy + dy;
            if (jx < 0 || jx >= nsx || jy < 0 || jy >= nsy) return T(0);
            const int q = jy * nsx + jx;
            const T v = rhs(jy, jx) * invd[q];
            return TRANS ? cpk[q] * v : v;
        };
        const T nb = ax * (y1(-1, 0) + y1(1, 0)) + ay * (y1(0, -1) + y1(0, 1));
        y[p] = (c - (TRANS ? nb : cpk[p] * nb)) * invd[p];
    }
}

// Further sweeps: y_out = (c - coupling(y_in)) / d with c re-formed by rhs().
template <typename T, bool TRANS, typename RHS>
__device__ __forceinline__ void jacobi_more(const StreamArgs &a, const RowUnit &u, const T *invd,
                                            const T *cpk, const T *yin, T *yout, RHS rhs)
{
    const DevProblem &P = a.P;
    const int nsx = P.nsx, nsy = P.nsy, iy = u.iy;
    const T ax = T(P.idx2), ay = T(P.idy2);
    for (int ix = threadIdx.x; ix < nsx; ix += blockDim.x) {
        const int p = iy * nsx + ix;
        auto yv = [&](int dx, int dy) -> T {
            const int jx = ix + dx, jy = iy + dy;
            if (jx < 0 || jx >= nsx || jy < 0 || jy >= nsy) return T(0);
            const int q = jy * nsx + jx;
            return TRANS ? cpk[q] * yin[q] : yin[q];
        };
        const T nb = ax * (yv(-1, 0) + yv(1, 0)) + ay * (yv(0, -1) + yv(0, 1));
        yout[p] = (rhs(iy, ix) - (TRANS ? nb : cpk[p] * nb)) * invd[p];
    }
}

// F_x solve: c = sgn (b1 - h B v3) (sgn = -1 in the Schur iterations, where
// c = h B v3 - b1; +1 in the final block). pass 0: first two sweeps into y5;
// pass s >= 1: sweep s + 2 from y5 / ytmp (ping-pong by parity).
template <typename T>
__global__ void __launch_bounds__(256) k_st_jf(const StreamArgs a, int sgn, int use_v3, int pass)
{
    const RowUnit u = row_unit(a);
    if (!u.ok || !a.work[u.b]) return;
    const int n = a.P.nsx * a.P.nsy;
    const size_t bi = (size_t)u.b * a.P.N + u.i;
    const T *b1 = reinterpret_cast<const T *>(a.b1) + bi * n;
    const T *invd = reinterpret_cast<const T *>(a.invd) + bi * n;
    const T *cpk = reinterpret_cast<const T *>(a.cpk) + bi * n;
    T *y5 = reinterpret_cast<T *>(a.y5) + bi * n, *yt = reinterpret_cast<T *>(a.ytmp) + bi * n;
    const T h = T(a.P.h);
    auto rhs = [&](int jy, int jx) -> T {
        const T bv = use_v3 ? T(bsep_at(a, bi, jy, jx)) : T(0);
        const T v = b1[jy * a.P.nsx + jx] - h * bv;
        return sgn > 0 ? v : -v;
    };
    if (pass == 0) {
        jacobi_first<T, false>(a, u, bi, a.n_sw, invd, cpk, y5, rhs);
    } else {
        // sweeps 3, 4, ...: odd passes read y5 and write ytmp, even passes back
        const T *yin = (pass & 1) ? y5 : yt;
        T *yout = (pass & 1) ? yt : y5;
        jacobi_more<T, false>(a, u, invd, cpk, yin, yout, rhs);
    }
}

// c' = sgn b2 - A_xx y5 (sgn = -1 in the Schur iterations: c' = -b2 - A_xx y5),
// A_xx y = h ((q - 2 c0 g2) y + g2 N(y) + N(g2 y)). y5 is the F_x solve's
// result (in ytmp when its last pass was odd).
template <typename T>
__global__ void __launch_bounds__(256) k_st_axx(const StreamArgs a, int sgn, int y_in_tmp)
{
    const RowUnit u = row_unit(a);
    if (!u.ok || !a.work[u.b]) return;
    const DevProblem &P = a.P;
    const int nsx = P.nsx, nsy = P.nsy, n = nsx * nsy, iy = u.iy;
    const size_t bi = (size_t)u.b * P.N + u.i;
    const T *y = reinterpret_cast<const T *>(y_in_tmp ? a.ytmp : a.y5) + bi * n;
    const T *g2 = reinterpret_cast<const T *>(a.g2) + bi * n;
    const T *b2 = reinterpret_cast<const T *>(a.b2) + bi * n;
    T *cp = reinterpret_cast<T *>(a.cp) + bi * n;
    const T ax = T(P.idx2), ay = T(P.idy2), h = T(P.h), q = T(P.q), c0 = T(P.c0);
    for (int ix = threadIdx.x; ix < nsx; ix += blockDim.x) {
        const int p = iy * nsx + ix;
        auto v = [&](int dx, int dy, bool scaled) -> T {
            const int jx = ix + dx, jy = iy + dy;
            if (jx < 0 || jx >= nsx || jy < 0 || jy >= nsy) return T(0);
            const int qq = jy * nsx + jx;
            return scaled ? g2[qq] * y[qq] : y[qq];
        };
        const T n1 = ax * (v(-1, 0, false) + v(1, 0, false)) + ay * (v(0, -1, false) + v(0, 1, false));
        const T n2 = ax * (v(-1, 0, true) + v(1, 0, true)) + ay * (v(0, -1, true) + v(0, 1, true));
        const T Ay = h * ((q - T(2) * c0 * g2[p]) * y[p] + g2[p] * n1 + n2);
        cp[p] = (sgn > 0 ? b2[p] : -b2[p]) - Ay;
    }
}

// F_x^T solve of c' into y4 (pass as in k_st_jf, ping-pong with y4tmp); on the
// last pass optionally the row partials of B^T y4, and in the final block the
// update of x and lambda into the other iterate buffer.
template <typename T>
__global__ void __launch_bounds__(256) k_st_jft(const StreamArgs a, int pass, int last_pass,
                                                int partials, int update, int y5_in_tmp)
{
    __shared__ double sh[kMaxWaves];
    const RowUnit u = row_unit(a);
    if (!u.ok || !a.work[u.b]) return;
    const DevProblem &P = a.P;
    const int nsx = P.nsx, n = nsx * P.nsy, iy = u.iy;
    const size_t bi = (size_t)u.b * P.N + u.i;
    const T *invd = reinterpret_cast<const T *>(a.invd) + bi * n;
    const T *cpk = reinterpret_cast<const T *>(a.cpk) + bi * n;
    const T *cp = reinterpret_cast<const T *>(a.cp) + bi * n;
    T *y4 = reinterpret_cast<T *>(a.y4) + bi * n, *yt = reinterpret_cast<T *>(a.y4tmp) + bi * n;
    auto rhs = [&](int jy, int jx) -> T { return cp[jy * nsx + jx]; };
    T *res = y4;
    if (pass == 0) {
        jacobi_first<T, true>(a, u, bi, a.n_sw, invd, cpk, y4, rhs);
    } else {
        const T *yin = (pass & 1) ? y4 : yt;
        res = (pass & 1) ? yt : y4;
        jacobi_more<T, true>(a, u, invd, cpk, yin, res, rhs);
    }
    if (!last_pass) return;
    __syncthreads();   // this thread's own results are read back below
    if (partials) {
        double tl[kMaxLx];
        for (int q = 0; q < P.lx; ++q) tl[q] = 0.0;
        for (int ix = threadIdx.x; ix < nsx; ix += blockDim.x) {
            const double yv = double(res[iy * nsx + ix]);
            for (int q = 0; q < P.lx; ++q) tl[q] += a.gx[q * nsx + ix] * yv;
        }
        const size_t ru = bi * P.nsy + iy;
        for (int q = 0; q < P.lx; ++q) {
            const double s = block_sum(tl[q], sh);
            if (threadIdx.x == 0) a.rowt[ru * kMaxLx + q] = s;
        }
    }
    if (update) {
        const int cur = a.st[u.b].j & 1, nxt = cur ^ 1;
        const T *y5 = reinterpret_cast<const T *>(y5_in_tmp ? a.ytmp : a.y5) + bi * n;
        const double *x = a.X[cur] + bi * n, *lam = a.LAM[cur] + bi * n;
        double *xn = a.X[nxt] + bi * n, *ln = a.LAM[nxt] + bi * n;
        for (int ix = threadIdx.x; ix < nsx; ix += blockDim.x) {
            const int p = iy * nsx + ix;
            xn[p] = x[p] - double(y5[p]);
            ln[p] = lam[p] - double(res[p]);
        }
        if (iy == 0) {
            const double *uc = a.U[cur] + bi * P.m;
            double *un = a.U[nxt] + bi * P.m;
            for (int j = threadIdx.x; j < P.m; j += blockDim.x) un[j] = uc[j] - a.v3[bi * P.m + j];
        }
    }
}

// v3 = (K^u + h B^T y4) / (h r + gamma) per stage (T arithmetic as in the
// fused kernel). One workgroup (64 threads) per stage.
template <typename T>
__global__ void k_st_v3(const StreamArgs a)
{
    const int bi = blockIdx.x;
    if (bi >= a.count * a.P.N) return;
    const int b = bi / a.P.N;
    if (!a.work[b]) return;
    const T auu = T(a.P.h * a.P.r + a.P.gamma), h = T(a.P.h);
    for (int j = threadIdx.x; j < a.P.m; j += blockDim.x) {
        const T bt = T(bt_from_rows(a, bi, j));
        a.v3[(size_t)bi * a.P.m + j] = double((T(a.kun[(size_t)bi * a.P.m + j]) + h * bt) / auu);
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
    if (prec == kModeFp32) {
        k.bsep = (const void *)&k_st_bsep<kModeFp32>;
        k.stage = (const void *)&k_st_stage<kModeFp32>;
        k.res = (const void *)&k_st_res<float>;
        k.decide = (const void *)&k_st_decide<kModeFp32>;
        k.jf = (const void *)&k_st_jf<float>;
        k.axx = (const void *)&k_st_axx<float>;
        k.jft = (const void *)&k_st_jft<float>;
        k.v3 = (const void *)&k_st_v3<float>;
    } else {
        k.bsep = (const void *)&k_st_bsep<kModeFp64>;
        k.stage = (const void *)&k_st_stage<kModeFp64>;
        k.res = (const void *)&k_st_res<double>;
        k.decide = (const void *)&k_st_decide<kModeFp64>;
        k.jf = (const void *)&k_st_jf<double>;
        k.axx = (const void *)&k_st_axx<double>;
        k.jft = (const void *)&k_st_jft<double>;
        k.v3 = (const void *)&k_st_v3<double>;
    }
    return k;
}

}  // namespace nmpc
