// nmpc_kernels.hip -- gfx950 kernels of the double-layer Jacobi NMPC solver.
//
// One workgroup owns one (instance, stage) unit of one upper iteration
// (eq. 1st_jacobi: every stage block is solved from S^k alone, so all units of
// an iteration are independent). Inside the workgroup the stage grid is held
// in registers: lane = grid column ix (nsx <= 64), wave w = a band of R rows.
// x-neighbours come from the adjacent lanes by cross-lane shuffles, y-neighbours
// from the lane's own registers, and only the band-edge rows go through LDS.
//
// Per unit and upper iteration the kernel fuses:
//   1. the KKT rows K_i (Sec. 3.2) in FP64 and their inf-norms, accumulated
//      per instance with integer atomic max on the IEEE bit patterns;
//   2. the lower layer (Sec. 4.3): stage coefficients, n_schur Schur input
//      iterations with diagonal A_uu (Sec. 5.2), each F_x / F_x^T solve by
//      n_sweep point-Jacobi sweeps from zero (Lemma lemma_jaco), then the
//      saddle solve of eq. step2 / eq. coff;
//   3. the update S^{k+1} = S^k - ds (alpha = 1), written to the other buffer.
// The lower layer runs in T (double, or float for the FP32-sweep variant);
// S, K, the norms and the convergence test are always FP64.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmpc_device.h"

namespace nmpc {

__device__ __forceinline__ unsigned long long abits(double v)
{
    return (unsigned long long)__double_as_longlong(fabs(v));
}
__device__ __forceinline__ double bits2d(unsigned long long b)
{
    return __longlong_as_double((long long)b);
}
__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b)
{
    return a > b ? a : b;
}

template <int M>
struct Pow2 {
    static constexpr int v = M <= 1 ? 1 : M <= 2 ? 2 : M <= 4 ? 4 : M <= 8 ? 8 : M <= 16 ? 16
                           : M <= 32 ? 32 : 64;
    static constexpr int lg = v == 1 ? 0 : v == 2 ? 1 : v == 4 ? 2 : v == 8 ? 3 : v == 16 ? 4
                            : v == 32 ? 5 : 6;
};

// Shared memory of one workgroup.
struct Lds {
    double edge[2][2][kMaxWaves][kWave];   // [flip][top,bottom][wave][lane]
    double gy[kMaxLy][kMaxRows];            // gy[b][iy]
    double uvec[kMaxM];                     // u_i
    double v3[kMaxM];                       // Schur iterate (input correction)
    double kun[kMaxM];                      // K^u_i
    double red[kMaxWaves][kMaxM];           // per-wave partial sums
    unsigned long long nrm[kMaxWaves][4];   // per-wave partial maxima
};

struct Ctx {
    Lds *L;
    int lane, w, W, flip;
    double ax, ay;   // 1/dx^2, 1/dy^2
};

// Neighbour sum N(v)_p = (v_l + v_r)/dx^2 + (v_u + v_d)/dy^2 with zero values
// off the grid (the Laplacian is L v = N(v) - (2/dx^2 + 2/dy^2) v).
template <typename V, int R>
__device__ __forceinline__ void nbsum(const V (&v)[R], V (&o)[R], Ctx &c)
{
    V above = V(0), below = V(0);
    if (c.W > 1) {
        V *top = reinterpret_cast<V *>(&c.L->edge[c.flip][0][0][0]);
        V *bot = reinterpret_cast<V *>(&c.L->edge[c.flip][1][0][0]);
        top[c.w * kWave + c.lane] = v[0];
        bot[c.w * kWave + c.lane] = v[R - 1];
        __syncthreads();
        if (c.w > 0) above = bot[(c.w - 1) * kWave + c.lane];
        if (c.w + 1 < c.W) below = top[(c.w + 1) * kWave + c.lane];
        c.flip ^= 1;
    }
    const V ax = V(c.ax), ay = V(c.ay);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        V lf = __shfl_up(v[r], 1, kWave);
        V rt = __shfl_down(v[r], 1, kWave);
        lf = c.lane == 0 ? V(0) : lf;
        rt = c.lane == kWave - 1 ? V(0) : rt;
        V up = r > 0 ? v[r - 1] : above;
        V dn = r < R - 1 ? v[r + 1] : below;
        o[r] = ax * (lf + rt) + ay * (up + dn);
    }
}

// Reduce per-lane arrays over the 64 lanes of a wave, starting after FIRST
// halving steps already done by the caller (a holds MP values). On return,
// lane l holds the total of element (l >> (6 - log2(MP) - FIRST)): each
// halving step trades the half a lane does not keep with its partner, so the
// exchange volume is about the element count instead of 6x it.
template <int MP, int FIRST, typename V>
__device__ __forceinline__ V wave_reduce_scatter_from(V (&a)[MP], int lane)
{
    constexpr int LG = Pow2<MP>::lg;
#pragma unroll
    for (int s = 0; s < LG; ++s) {
        const int mask = 32 >> (s + FIRST);
        const int half = MP >> (s + 1);
        const bool hi = (lane & mask) != 0;
#pragma unroll
        for (int j = 0; j < half; ++j) {
            V send = hi ? a[j] : a[j + half];
            V keep = hi ? a[j + half] : a[j];
            a[j] = keep + __shfl_xor(send, mask, kWave);
        }
    }
    V s = a[0];
#pragma unroll
    for (int mask = 32 >> (LG + FIRST); mask >= 1; mask >>= 1) s += __shfl_xor(s, mask, kWave);
    return s;
}

__device__ __forceinline__ unsigned long long wave_max64(unsigned long long v)
{
#pragma unroll
    for (int mask = 32; mask >= 1; mask >>= 1) v = umax64(v, __shfl_xor(v, mask, kWave));
    return v;
}

// (B v)_p = sum_b gy[b][iy] sum_a gx[a][ix] v[b*LX + a]; v in LDS (double).
template <typename V, int R, int LX, int LY>
__device__ __forceinline__ void b_apply(const double *vs, const double (&gxr)[LX], Ctx &c,
                                        V (&o)[R])
{
    V s[LY];
#pragma unroll
    for (int b = 0; b < LY; ++b) {
        V acc = V(0);
#pragma unroll
        for (int a = 0; a < LX; ++a) acc += V(gxr[a]) * V(vs[b * LX + a]);
        s[b] = acc;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int iy = c.w * R + r;
        V acc = V(0);
#pragma unroll
        for (int b = 0; b < LY; ++b) acc += V(c.L->gy[b][iy]) * s[b];
        o[r] = acc;
    }
}

// out[j] = (B^T y)_j for j < M, left in L->red[0][j] (double); all threads
// synchronized on return. Per lane: t_b = sum_r gy[b][iy_r] y_r, then the
// products gx[a][ix] t_b are formed inside the first halving step of the
// cross-lane reduction (so the M-wide product array is never held).
template <typename V, int R, int LX, int LY>
__device__ __forceinline__ void bt_reduce(const V (&y)[R], const double (&gxr)[LX], Ctx &c,
                                          int tid, int M)
{
    constexpr int MP = Pow2<LX * LY>::v;
    constexpr int MM = LX * LY;
    V t[LY];
#pragma unroll
    for (int b = 0; b < LY; ++b) {
        V acc = V(0);
#pragma unroll
        for (int r = 0; r < R; ++r) acc += V(c.L->gy[b][c.w * R + r]) * y[r];
        t[b] = acc;
    }
    V e;
    if constexpr (MP == 1) {
        e = V(gxr[0]) * t[0];
#pragma unroll
        for (int mask = 32; mask >= 1; mask >>= 1) e += __shfl_xor(e, mask, kWave);
    } else {
        constexpr int HALF = MP / 2;
        V a[HALF];
        const bool hi = (c.lane & 32) != 0;
#pragma unroll
        for (int j = 0; j < HALF; ++j) {
            const int jl = j, jh = j + HALF;
            const V pl = jl < MM ? V(gxr[jl % LX]) * t[jl / LX] : V(0);
            const V ph = jh < MM ? V(gxr[jh % LX]) * t[jh / LX] : V(0);
            const V send = hi ? pl : ph;
            const V keep = hi ? ph : pl;
            a[j] = keep + __shfl_xor(send, 32, kWave);
        }
        e = wave_reduce_scatter_from<HALF, 1>(a, c.lane);
    }
    constexpr int SH = 6 - Pow2<MP>::lg;
    if ((c.lane & ((1 << SH) - 1)) == 0) c.L->red[c.w][c.lane >> SH] = double(e);
    __syncthreads();
    if (tid < M) {
        V s = V(0);
        for (int ww = 0; ww < c.W; ++ww) s += V(c.L->red[ww][tid]);
        c.L->red[0][tid] = double(s);   // only thread tid touches column tid
    }
    __syncthreads();
}

// ----------------------------------------------------------- lower layer

template <typename T, int R>
struct StageCoef {
    T invd[R];   // 1 / diag(F_x)
    T cpk[R];    // h k(x_p): F_x off-diagonal = h k_p / dx^2
    T g2[R];     // k' lambda_p (enters A_xx)
};

// n_sw point-Jacobi sweeps on F_x y = c from y = 0.
template <typename T, int R>
__device__ __forceinline__ void jac_f(const T (&cc)[R], T (&y)[R], const StageCoef<T, R> &K,
                                      int n_sw, Ctx &c)
{
#pragma unroll
    for (int r = 0; r < R; ++r) y[r] = cc[r] * K.invd[r];
    for (int s = 1; s < n_sw; ++s) {
        T nb[R];
        nbsum<T, R>(y, nb, c);
#pragma unroll
        for (int r = 0; r < R; ++r) y[r] = (cc[r] - K.cpk[r] * nb[r]) * K.invd[r];
    }
}

// n_sw point-Jacobi sweeps on F_x^T y = c from y = 0; (F_x^T)_{pq} = h k_q / dx^2.
template <typename T, int R>
__device__ __forceinline__ void jac_ft(const T (&cc)[R], T (&y)[R], const StageCoef<T, R> &K,
                                       int n_sw, Ctx &c)
{
#pragma unroll
    for (int r = 0; r < R; ++r) y[r] = cc[r] * K.invd[r];
    for (int s = 1; s < n_sw; ++s) {
        T z[R], nb[R];
#pragma unroll
        for (int r = 0; r < R; ++r) z[r] = K.cpk[r] * y[r];
        nbsum<T, R>(z, nb, c);
#pragma unroll
        for (int r = 0; r < R; ++r) y[r] = (cc[r] - nb[r]) * K.invd[r];
    }
}

// A_xx y = h (q y + k' (diag(lam) L + L diag(lam)) y)
//        = h ((q - 2 c0 g2) y + g2 N(y) + N(g2 y)).
template <typename T, int R>
__device__ __forceinline__ void axx_apply(const T (&y)[R], T (&o)[R], const StageCoef<T, R> &K,
                                          T h, T q, T c0, Ctx &c)
{
    T nb1[R], z[R], nb2[R];
    nbsum<T, R>(y, nb1, c);
#pragma unroll
    for (int r = 0; r < R; ++r) z[r] = K.g2[r] * y[r];
    nbsum<T, R>(z, nb2, c);
#pragma unroll
    for (int r = 0; r < R; ++r)
        o[r] = h * ((q - T(2) * c0 * K.g2[r]) * y[r] + K.g2[r] * nb1[r] + nb2[r]);
}

// ------------------------------------------------------------- the kernel

struct Decision {
    bool work;     // evaluate and update this kernel
    int j;         // index of the iterate evaluated (S^j)
    bool fp32;     // lower layer in FP32
};

// Per-instance state machine. All workgroups of an instance compute the same
// decision from data that no one writes during this kernel (the state slot of
// this kernel's parity and the residual slot of the previous kernel); the
// stage-0 workgroup publishes the next state into the other parity slot.
__device__ Decision decide(const IterArgs &a, int b, int stage, int k, int tid)
{
    InstState s = a.st[(k & 1) * a.B + b];
    InstState ns = s;
    Decision d{false, 0, false};
    int fin = -1, fin_iter = 0;
    double rs = 0.0, rp = 0.0;
    if (s.status == kActive) {
        const int jprev = k - 1 - s.off;
        if (k == 0 || jprev < 0) {
            d.work = true;
            d.j = 0;
        } else {
            const int slot = (k - 1) % 3;
            rs = bits2d(a.racc[slot * a.B + b]);
            rp = bits2d(a.pacc[slot * a.B + b]);
            if (!(rs <= 1.7976931348623157e308)) {          // NaN or Inf
                fin = kStatusNonfinite;
                fin_iter = jprev;
            } else if (rs <= a.tol) {
                if (s.mode == 1) {                           // FP32 phase done:
                    ns.mode = 0;                             // redo S^jprev in FP64
                    ns.pending = 1;
                    ns.off = s.off + 1;
                    d.work = true;
                    d.j = jprev;
                } else if (s.pending) {                      // FP64 correction step
                    ns.pending = 0;
                    d.work = true;
                    d.j = jprev + 1;
                } else {
                    fin = kStatusOk;
                    fin_iter = jprev;
                }
            } else if (jprev >= a.max_iter) {
                fin = kStatusNoconv;
                fin_iter = jprev;
            } else {
                d.work = true;
                d.j = jprev + 1;
            }
        }
        d.fp32 = d.work && ns.mode == 1;
        if (d.fp32) ns.f32 = s.f32 + 1;
        if (fin >= 0) ns.status = fin;
    }
    if (stage == 0 && tid == 0) {
        a.st[((k + 1) & 1) * a.B + b] = ns;
        if (fin >= 0) {
            a.iters[b] = fin_iter;
            a.rfin[2 * b] = rs;
            a.rfin[2 * b + 1] = rp;
            atomicAdd(a.ctr + 2, 1);
        }
        if (d.work) {   // this kernel accumulates slot k%3; clear the next one
            a.racc[((k + 1) % 3) * a.B + b] = 0ull;
            a.pacc[((k + 1) % 3) * a.B + b] = 0ull;
        }
    }
    return d;
}

template <typename T, int R, int LX, int LY>
__device__ __forceinline__ void stage_body(const IterArgs &a, Ctx &c, const double (&gxr)[LX],
                                           int b, int i, int j, int slot, int tid)
{
    const DevProblem &P = a.P;
    constexpr int M = LX * LY;
    const int n = P.n, lane = c.lane;
    const int cur = j & 1, nxt = cur ^ 1;
    const size_t unit = (size_t)b * P.N + i;

    // ---- loads (FP64): x_i, lam_i, u_i now; x_{i-1}, lam_{i+1}, xref_i when used
    double xc[R], lc[R];
    const double *Xc = a.X[cur] + unit * n;
    const double *Lc = a.LAM[cur] + unit * n;
    const double *Xp = (i == 0) ? a.x0 + (size_t)b * n : a.X[cur] + (unit - 1) * n;
    const double *Ln = a.LAM[cur] + (unit + 1) * n;
    const double *Xr = a.xref + (size_t)b * a.xref_inst_stride + (size_t)i * a.xref_stage_stride;
    const bool last = (i == P.N - 1);
    int pidx[R];
    bool pval[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int iy = c.w * R + r;
        pval[r] = lane < P.nsx && iy < P.nsy;
        pidx[r] = iy * P.nsx + lane;
        xc[r] = pval[r] ? Xc[pidx[r]] : 0.0;
        lc[r] = pval[r] ? Lc[pidx[r]] : 0.0;
    }
    if (tid < M) c.L->uvec[tid] = a.U[cur][unit * M + tid];

    // ---- KKT rows (FP64)
    //   K^lam = lam_{i+1} - lam + h (q (x - xref) + L(k lam) + k' (L x) lam)
    //   K^x   = x_{i-1} - x + h (k L x + B u)
    const double h = P.h, kp = P.k0 * P.k1;
    double Lx[R], KX[R], KL[R];
    nbsum<double, R>(xc, Lx, c);   // (its LDS barrier also publishes uvec)
    {
        double g[R], Lg[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            Lx[r] -= P.c0 * xc[r];
            g[r] = P.k0 * (1.0 + P.k1 * xc[r]) * lc[r];
        }
        nbsum<double, R>(g, Lg, c);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double ln = (pval[r] && !last) ? Ln[pidx[r]] : 0.0;
            const double xr = pval[r] ? Xr[pidx[r]] : 0.0;
            // off-grid lanes/rows see a nonzero stencil of their valid neighbour:
            // their rows do not exist and are zeroed (norms, right-hand sides)
            KL[r] = pval[r] ? ln - lc[r] + h * (P.q * (xc[r] - xr) + (Lg[r] - P.c0 * g[r]) +
                                                kp * Lx[r] * lc[r])
                            : 0.0;
        }
    }
    if (c.W == 1) __syncthreads();   // uvec visible without an LDS stencil barrier
    {
        double Bu[R];
        b_apply<double, R, LX, LY>(c.L->uvec, gxr, c, Bu);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double xp = pval[r] ? Xp[pidx[r]] : 0.0;
            const double kk = P.k0 * (1.0 + P.k1 * xc[r]);
            KX[r] = pval[r] ? xp - xc[r] + h * (kk * Lx[r] + Bu[r]) : 0.0;
        }
    }
    unsigned long long mx = 0, ml = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        mx = umax64(mx, abits(KX[r]));
        ml = umax64(ml, abits(KL[r]));
    }
    bt_reduce<double, R, LX, LY>(lc, gxr, c, tid, M);
    unsigned long long mu = 0;
    if (tid < M) {
        const double ku = h * (P.r * c.L->uvec[tid] + c.L->red[0][tid]);   // u~ = u: no gamma term
        c.L->kun[tid] = ku;
        c.L->v3[tid] = 0.0;
        mu = abits(ku);
    }
    mx = wave_max64(mx);
    ml = wave_max64(ml);
    mu = wave_max64(mu);
    if (lane == 0) {
        c.L->nrm[c.w][0] = mx;
        c.L->nrm[c.w][1] = ml;
        c.L->nrm[c.w][2] = mu;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long ax = 0, al = 0, au = 0;
        for (int ww = 0; ww < c.W; ++ww) {
            ax = umax64(ax, c.L->nrm[ww][0]);
            al = umax64(al, c.L->nrm[ww][1]);
            au = umax64(au, c.L->nrm[ww][2]);
        }
        const double dx_ = bits2d(ax), dl_ = bits2d(al), du_ = bits2d(au);
        double rp = dx_ > du_ ? dx_ : du_;
        rp = rp > dl_ ? rp : dl_;
        double rs = dx_, su = du_ / (h * P.r), sl = dl_ / h;
        rs = rs > su ? rs : su;
        rs = rs > sl ? rs : sl;
        // NaN-propagating: any non-finite row makes both norms non-finite
        const bool bad = (ax >= 0x7FF0000000000000ull) || (al >= 0x7FF0000000000000ull) ||
                         (au >= 0x7FF0000000000000ull);
        if (bad) { rs = __longlong_as_double(0x7FF8000000000000ll); rp = rs; }
        atomicMax(a.racc + (size_t)slot * a.B + b, abits(rs));
        atomicMax(a.pacc + (size_t)slot * a.B + b, abits(rp));
    }
    if (a.residual_only) return;

    // ---- lower layer (T)
    StageCoef<T, R> K;
    T b1[R], b2[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int iy = c.w * R + r;
        const bool v = lane < P.nsx && iy < P.nsy;
        const double kk = P.k0 * (1.0 + P.k1 * xc[r]);
        const double d = -1.0 - h * kk * P.c0 + h * kp * Lx[r];      // diag of F_x
        K.invd[r] = v ? T(1.0 / d) : T(0);
        K.cpk[r] = T(h * kk);
        K.g2[r] = T(kp * lc[r]);
        b1[r] = T(KX[r]);
        b2[r] = T(KL[r]);
    }
    const T hT = T(h), qT = T(P.q), c0T = T(P.c0);
    const double auu = h * P.r + P.gamma;
    T y5[R], y4[R], cc[R], Ay[R];
    for (int s = 0; s < a.n_schur; ++s) {
        if (s == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) cc[r] = -b1[r];
        } else {
            T Bv[R];
            b_apply<T, R, LX, LY>(c.L->v3, gxr, c, Bv);
#pragma unroll
            for (int r = 0; r < R; ++r) cc[r] = hT * Bv[r] - b1[r];
        }
        jac_f<T, R>(cc, y5, K, a.n_sw, c);
        axx_apply<T, R>(y5, Ay, K, hT, qT, c0T, c);
#pragma unroll
        for (int r = 0; r < R; ++r) cc[r] = -b2[r] - Ay[r];
        jac_ft<T, R>(cc, y4, K, a.n_sw, c);
        bt_reduce<T, R, LX, LY>(y4, gxr, c, tid, M);
        if (tid < M) {
            const T bt = T(c.L->red[0][tid]);
            c.L->v3[tid] = double((T(c.L->kun[tid]) + hT * bt) / T(auu));
        }
        __syncthreads();
    }
    {
        T Bv[R];
        b_apply<T, R, LX, LY>(c.L->v3, gxr, c, Bv);
#pragma unroll
        for (int r = 0; r < R; ++r) cc[r] = b1[r] - hT * Bv[r];
    }
    jac_f<T, R>(cc, y5, K, a.n_sw, c);          // v2 = dx
    axx_apply<T, R>(y5, Ay, K, hT, qT, c0T, c);
#pragma unroll
    for (int r = 0; r < R; ++r) cc[r] = b2[r] - Ay[r];
    jac_ft<T, R>(cc, y4, K, a.n_sw, c);         // v1 = dlam

    // ---- update S^{j+1} = S^j - ds (FP64)
    double *Xn = a.X[nxt] + unit * n;
    double *Lnw = a.LAM[nxt] + unit * n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int iy = c.w * R + r;
        if (lane < P.nsx && iy < P.nsy) {
            const int p = iy * P.nsx + lane;
            Xn[p] = xc[r] - double(y5[r]);
            Lnw[p] = lc[r] - double(y4[r]);
        }
    }
    if (tid < M) a.U[nxt][unit * M + tid] = c.L->uvec[tid] - c.L->v3[tid];
}

template <int PREC, int R, int LX, int LY>
__global__ void __launch_bounds__(kWave * kMaxWaves) k_iterate(const IterArgs a)
{
    __shared__ Lds L;
    const int tid = threadIdx.x;
    Ctx c;
    c.L = &L;
    c.lane = tid & (kWave - 1);
    c.w = tid / kWave;
    c.W = blockDim.x / kWave;
    c.flip = 0;
    c.ax = a.P.idx2;
    c.ay = a.P.idy2;

    const int k = a.residual_only ? 0 : *(volatile const int *)(a.ctr);
    // XCD-aware unit order: consecutive workgroup ids go to different XCDs, so
    // give each XCD a contiguous run of units (neighbouring stages of one
    // instance then share that XCD's L2 for the x_{i-1} / lambda_{i+1} reads).
    const int bid = blockIdx.x;
    const int unit = (bid & 7) * a.per_xcd + (bid >> 3);
    if (unit < a.units) {
        const int b = unit / a.P.N, i = unit % a.P.N;
        Decision d;
        if (a.residual_only) {
            d.work = true; d.j = 0; d.fp32 = false;
        } else {
            d = decide(a, b, i, k, tid);
        }
        if (d.work) {
            for (int t = tid; t < LY * kMaxRows; t += blockDim.x) {
                const int bb = t / kMaxRows, iy = t % kMaxRows;
                L.gy[bb][iy] = iy < a.P.nsy ? a.gy[bb * a.P.nsy + iy] : 0.0;
            }
            double gxr[LX];
#pragma unroll
            for (int aa = 0; aa < LX; ++aa)
                gxr[aa] = c.lane < a.P.nsx ? a.gx[aa * a.P.nsx + c.lane] : 0.0;
            const int slot = a.residual_only ? 0 : k % 3;
            if (tid == 0 && !a.residual_only) atomicAdd(a.work_units, 1ull);
            if (PREC == 1 && d.fp32)
                stage_body<float, R, LX, LY>(a, c, gxr, b, i, d.j, slot, tid);
            else
                stage_body<double, R, LX, LY>(a, c, gxr, b, i, d.j, slot, tid);
        }
    }
    if (a.residual_only) return;
    // Last workgroup to finish advances the device iteration counter, so a
    // captured sequence of launches needs no per-launch argument.
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(a.wgdone, 1u);
        if (prev == gridDim.x - 1) {
            atomicExch(a.wgdone, 0u);
            atomicAdd(a.ctr, 1);
            __threadfence();
        }
    }
}

// S^0 into buffer 0: cold (x_i = x0, u_i = 0, lam_i = 0) or copied warm start.
__global__ void k_init(const InitArgs a)
{
    const size_t nN = (size_t)a.count * a.N * a.n;
    const size_t mN = (size_t)a.count * a.N * a.m;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < nN; t += stride) {
        const size_t b = t / ((size_t)a.N * a.n), p = t % a.n;
        a.X[t] = a.wx ? a.wx[t] : a.x0[b * a.n + p];
        a.LAM[t] = a.wl ? a.wl[t] : 0.0;
    }
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < mN; t += stride)
        a.U[t] = a.wu ? a.wu[t] : 0.0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)a.count;
         t += stride) {
        InstState s;
        s.status = kActive; s.mode = a.mode; s.off = 0; s.pending = 0; s.f32 = 0;
        a.st[t] = s;
        a.st[a.B + t] = s;
        for (int q = 0; q < 3; ++q) {
            a.racc[q * a.B + t] = 0ull;
            a.pacc[q * a.B + t] = 0ull;
        }
        a.iters[t] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctr[0] = 0;
        a.ctr[2] = 0;
        *a.wgdone = 0u;
    }
}

// Copy each instance's returned iterate (buffer iters[b] & 1) out.
__global__ void k_output(const OutArgs a)
{
    const size_t w = (size_t)a.N * a.n, wm = (size_t)a.N * a.m;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)a.count * w;
         t += stride) {
        const int b = (int)(t / w);
        const int buf = a.iters[b] & 1;
        a.ox[t] = a.X[buf][t];
        a.ol[t] = a.LAM[buf][t];
    }
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)a.count * wm;
         t += stride) {
        const int b = (int)(t / wm);
        a.ou[t] = a.U[a.iters[b] & 1][t];
    }
}

// ------------------------------------------------------ instantiation table

#define NMPC_INST(P, R, LX, LY) \
    if (prec == P && rows == R && lx == LX && ly == LY) return (const void *)&k_iterate<P, R, LX, LY>;

const void *iterate_kernel(int prec, int rows, int lx, int ly)
{
#define NMPC_ROWS(P, LX, LY) NMPC_INST(P, 1, LX, LY) NMPC_INST(P, 2, LX, LY) NMPC_INST(P, 4, LX, LY)
    NMPC_ROWS(0, 1, 1)
    NMPC_ROWS(1, 1, 1)
    NMPC_ROWS(0, 2, 1)
    NMPC_ROWS(1, 2, 1)
    NMPC_ROWS(0, 2, 2)
    NMPC_ROWS(1, 2, 2)
    NMPC_ROWS(0, 4, 4)
    NMPC_ROWS(1, 4, 4)
#undef NMPC_ROWS
    return nullptr;
}
#undef NMPC_INST

const void *init_kernel() { return (const void *)&k_init; }
const void *output_kernel() { return (const void *)&k_output; }

}  // namespace nmpc
