// nmpc_kernels.hip -- gfx950 kernels of the double-layer Jacobi NMPC solver.
//
// One workgroup owns one (instance, stage) unit of one upper iteration
// (eq. 1st_jacobi: every stage block is solved from S^k alone, so all units of
// an iteration are independent). Inside the workgroup the stage grid is held
// in registers as tiles: 16 lanes span a grid row, each lane owning CX
// consecutive columns and RY consecutive rows; the four 16-lane rows of a
// wave and the waves of the workgroup stack downwards. Stencil neighbours
// inside a tile are registers, the left/right tile edges come from the
// adjacent lane by DPP row shifts (VALU, zero-filled at the row ends, which is
// the Dirichlet value), and only the top/bottom tile rows pass through LDS.
//
// Per unit and upper iteration the kernel fuses:
//   1. the KKT rows K_i (Sec. 3.2) in FP64 and their inf-norms, accumulated
//      per instance with integer atomic max on the IEEE bit patterns;
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

// DPP row shifts: lane l of a 16-lane row receives lane l-1 (shr) or l+1
// (shl) of the same row; the lane without a source receives 0.
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShl1 = 0x101;

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Per-thread geometry and workgroup scratch.
struct Ctx {
    unsigned char *lds;
    LdsOff off;
    int tid, lane, cl, w, W, G, GT, Gv, flip;
    double ax, ay;   // 1/dx^2, 1/dy^2
};

template <typename V>
__device__ __forceinline__ V *lds_ptr(const Ctx &c, size_t o) { return reinterpret_cast<V *>(c.lds + o); }

// Neighbour sum N(v)_p = (v_l + v_r)/dx^2 + (v_u + v_d)/dy^2 with zero values
// off the grid (the Laplacian is L v = N(v) - (2/dx^2 + 2/dy^2) v).
template <typename V, int CX, int RY>
__device__ __forceinline__ void nbsum(const V (&v)[RY][CX], V (&o)[RY][CX], Ctx &c)
{
    V above[CX], below[CX];
#pragma unroll
    for (int q = 0; q < CX; ++q) { above[q] = V(0); below[q] = V(0); }
    if (c.Gv > 1) {   // tile rows shared through LDS (double-buffered by flip)
        V *top = lds_ptr<V>(c, c.off.edge) + (size_t)c.flip * 2 * c.GT * 16 * CX;
        V *bot = top + (size_t)c.GT * 16 * CX;
        const int me = (c.G * 16 + c.cl) * CX;
#pragma unroll
        for (int q = 0; q < CX; ++q) { top[me + q] = v[0][q]; bot[me + q] = v[RY - 1][q]; }
        __syncthreads();
        if (c.G > 0) {
#pragma unroll
            for (int q = 0; q < CX; ++q) above[q] = bot[me - 16 * CX + q];
        }
        if (c.G + 1 < c.Gv) {
#pragma unroll
            for (int q = 0; q < CX; ++q) below[q] = top[me + 16 * CX + q];
        }
        c.flip ^= 1;
    }
    const V ax = V(c.ax), ay = V(c.ay);
#pragma unroll
    for (int t = 0; t < RY; ++t) {
        const V lin = dpp<kDppRowShr1>(v[t][CX - 1]);
        const V rin = dpp<kDppRowShl1>(v[t][0]);
#pragma unroll
        for (int q = 0; q < CX; ++q) {
            const V l = q > 0 ? v[t][q - 1] : lin;
            const V r = q < CX - 1 ? v[t][q + 1] : rin;
            const V u = t > 0 ? v[t - 1][q] : above[q];
            const V d = t < RY - 1 ? v[t + 1][q] : below[q];
            o[t][q] = ax * (l + r) + ay * (u + d);
        }
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
template <typename V>
__device__ __forceinline__ const V *gx_tab(const Ctx &c)
{
    return lds_ptr<V>(c, sizeof(V) == 8 ? c.off.gx : c.off.gxf);
}
template <typename V>
__device__ __forceinline__ const V *gy_tab(const Ctx &c)
{
    return lds_ptr<V>(c, sizeof(V) == 8 ? c.off.gy : c.off.gyf);
}

template <typename V, int CX, int RY, int LX, int LY, typename VS>
__device__ __forceinline__ void b_apply(const VS *vs, const Ctx &c, V (&o)[RY][CX])
{
    const V *gx = gx_tab<V>(c);
    const V *gy = gy_tab<V>(c);
    V s[LY][CX];
#pragma unroll
    for (int b = 0; b < LY; ++b)
#pragma unroll
        for (int q = 0; q < CX; ++q) {
            V acc = V(0);
#pragma unroll
            for (int a = 0; a < LX; ++a)
                acc += V(gx[a * 16 * CX + c.cl * CX + q]) * V(vs[b * LX + a]);
            s[b][q] = acc;
        }
#pragma unroll
    for (int t = 0; t < RY; ++t) {
        V gyr[LY];
#pragma unroll
        for (int b = 0; b < LY; ++b) gyr[b] = V(gy[b * c.GT * RY + c.G * RY + t]);
#pragma unroll
        for (int q = 0; q < CX; ++q) {
            V acc = V(0);
#pragma unroll
            for (int b = 0; b < LY; ++b) acc += gyr[b] * s[b][q];
            o[t][q] = acc;
        }
    }
}

// (B^T y)_j for j < M, left in red[j] (double); all threads synchronized on
// return. Per lane: column partials t_b = sum_t gy[b][iy_t] y_t, then the
// products with gx are formed inside the first halving step of the
// cross-lane reduction, then the waves' partials are summed.
template <typename V, int CX, int RY, int LX, int LY>
__device__ __forceinline__ void bt_reduce(const V (&y)[RY][CX], Ctx &c, int M)
{
    constexpr int MP = Pow2<LX * LY>::v;
    constexpr int MM = LX * LY;
    const V *gx = gx_tab<V>(c);
    const V *gy = gy_tab<V>(c);
    double *red = lds_ptr<double>(c, c.off.red);
    V tb[LY][CX];
#pragma unroll
    for (int b = 0; b < LY; ++b)
#pragma unroll
        for (int q = 0; q < CX; ++q) tb[b][q] = V(0);
#pragma unroll
    for (int t = 0; t < RY; ++t)
#pragma unroll
        for (int b = 0; b < LY; ++b) {
            const V gyv = V(gy[b * c.GT * RY + c.G * RY + t]);
#pragma unroll
            for (int q = 0; q < CX; ++q) tb[b][q] += gyv * y[t][q];
        }
    auto prod = [&](int j) -> V {
        V acc = V(0);
        if (j < MM) {
#pragma unroll
            for (int q = 0; q < CX; ++q) acc += V(gx[(j % LX) * 16 * CX + c.cl * CX + q]) * tb[j / LX][q];
        }
        return acc;
    };
    V e;
    if constexpr (MP == 1) {
        e = prod(0);
#pragma unroll
        for (int mask = 32; mask >= 1; mask >>= 1) e += __shfl_xor(e, mask, kWave);
    } else {
        constexpr int HALF = MP / 2;
        V a[HALF];
        const bool hi = (c.lane & 32) != 0;
#pragma unroll
        for (int j = 0; j < HALF; ++j) {
            const V pl = prod(j), ph = prod(j + HALF);
            const V send = hi ? pl : ph;
            const V keep = hi ? ph : pl;
            a[j] = keep + __shfl_xor(send, 32, kWave);
        }
        e = wave_reduce_scatter_from<HALF, 1>(a, c.lane);
    }
    constexpr int SH = 6 - Pow2<MP>::lg;
    if ((c.lane & ((1 << SH) - 1)) == 0) red[c.w * kMaxM + (c.lane >> SH)] = double(e);
    __syncthreads();
    if (c.tid < M) {
        V s = V(0);
        for (int ww = 0; ww < c.W; ++ww) s += V(red[ww * kMaxM + c.tid]);
        red[c.tid] = double(s);   // only thread tid touches column tid
    }
    __syncthreads();
}

// ----------------------------------------------------------- lower layer

template <typename T, int CX, int RY>
struct StageCoef {
    T invd[RY][CX];   // 1 / diag(F_x)
    T cpk[RY][CX];    // h k(x_p): F_x off-diagonal = h k_p / dx^2
    T g2[RY][CX];     // k' lambda_p (enters A_xx)
};

// n_sw point-Jacobi sweeps on F_x y = c from y = 0.
template <typename T, int CX, int RY>
__device__ __forceinline__ void jac_f(const T (&cc)[RY][CX], T (&y)[RY][CX],
                                      const StageCoef<T, CX, RY> &K, int n_sw, Ctx &c)
{
#pragma unroll
    for (int t = 0; t < RY; ++t)
#pragma unroll
        for (int q = 0; q < CX; ++q) y[t][q] = cc[t][q] * K.invd[t][q];
    for (int s = 1; s < n_sw; ++s) {
        T nb[RY][CX];
        nbsum<T, CX, RY>(y, nb, c);
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q)
                y[t][q] = (cc[t][q] - K.cpk[t][q] * nb[t][q]) * K.invd[t][q];
    }
}

// n_sw point-Jacobi sweeps on F_x^T y = c from y = 0; (F_x^T)_{pq} = h k_q / dx^2.
template <typename T, int CX, int RY>
__device__ __forceinline__ void jac_ft(const T (&cc)[RY][CX], T (&y)[RY][CX],
                                       const StageCoef<T, CX, RY> &K, int n_sw, Ctx &c)
{
#pragma unroll
    for (int t = 0; t < RY; ++t)
#pragma unroll
        for (int q = 0; q < CX; ++q) y[t][q] = cc[t][q] * K.invd[t][q];
    for (int s = 1; s < n_sw; ++s) {
        T z[RY][CX], nb[RY][CX];
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q) z[t][q] = K.cpk[t][q] * y[t][q];
        nbsum<T, CX, RY>(z, nb, c);
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q) y[t][q] = (cc[t][q] - nb[t][q]) * K.invd[t][q];
    }
}

// A_xx y = h (q y + k' (diag(lam) L + L diag(lam)) y)
//        = h ((q - 2 c0 g2) y + g2 N(y) + N(g2 y)).
template <typename T, int CX, int RY>
__device__ __forceinline__ void axx_apply(const T (&y)[RY][CX], T (&o)[RY][CX],
                                          const StageCoef<T, CX, RY> &K, T h, T q, T c0, Ctx &c)
{
    T nb1[RY][CX], z[RY][CX];
    nbsum<T, CX, RY>(y, nb1, c);
#pragma unroll
    for (int t = 0; t < RY; ++t)
#pragma unroll
        for (int p = 0; p < CX; ++p) z[t][p] = K.g2[t][p] * y[t][p];
    T nb2[RY][CX];
    nbsum<T, CX, RY>(z, nb2, c);
#pragma unroll
    for (int t = 0; t < RY; ++t)
#pragma unroll
        for (int p = 0; p < CX; ++p)
            o[t][p] = h * ((q - T(2) * c0 * K.g2[t][p]) * y[t][p] + K.g2[t][p] * nb1[t][p] +
                           nb2[t][p]);
}

// ------------------------------------------------------------- the kernel

struct Decision {
    bool work;     // evaluate and update in this kernel
    int j;         // index of the iterate evaluated (S^j)
    int slot;      // residual slot this evaluation accumulates into
};

// Per-instance state machine. All workgroups of an instance compute the same
// decision from data that no one writes during this kernel (the state slot of
// this kernel's parity and the per-stage residuals of the instance's previous
// evaluation, max-reduced here); the stage-0 workgroup publishes the next
// state into the other parity slot. PREC is this kernel's precision (kModeFp32 or kModeFp64); an
// instance in another mode waits for the kernel of its precision.
//   FP32 mode, test passed at S^j  -> REDO (FP32-active count decremented)
//   REDO (FP64 kernel)             -> re-evaluate S^j in FP64, owe one step
//   FP64 mode, test passed, owed   -> take the FP64 step S^{j+1}
//   FP64 mode, test passed         -> finished, S^j returned
template <int PREC>
__device__ Decision decide(const IterArgs &a, Ctx &c, int b, int stage, int k)
{
    const InstState s = a.st[(k & 1) * a.B + b];
    InstState ns = s;
    Decision d{false, 0, 0};
    int fin = -1;
    double rs = 0.0, rp = 0.0;
    if (s.status == kActive && s.e > 0) {
        // max over the stages' residuals of the previous evaluation (wave 0),
        // broadcast through LDS; NaN bit patterns order above every finite value
        unsigned long long *nrm = lds_ptr<unsigned long long>(c, c.off.nrm);
        if (c.w == 0) {
            const size_t base = ((size_t)((s.e - 1) % 3) * a.B + b) * a.P.N;
            unsigned long long ms = 0, mp = 0;
            for (int t = c.lane; t < a.P.N; t += kWave) {
                ms = umax64(ms, a.rst[base + t]);
                mp = umax64(mp, a.pst[base + t]);
            }
            ms = wave_max64(ms);
            mp = wave_max64(mp);
            if (c.lane == 0) { nrm[0] = ms; nrm[1] = mp; }
        }
        __syncthreads();
        rs = bits2d(nrm[0]);
        rp = bits2d(nrm[1]);
        __syncthreads();
    }
    if (s.status == kActive) {
        if (s.e == 0) {
            if (s.mode == PREC) { d.work = true; d.j = 0; }
        } else {
            if (!(rs <= 1.7976931348623157e308)) {            // NaN or Inf
                fin = kStatusNonfinite;
            } else if (s.mode == kModeFp64Redo) {
                if (PREC == kModeFp64) {
                    ns.mode = kModeFp64;
                    ns.pending = 1;
                    d.work = true;
                    d.j = s.j;
                }
            } else if (rs <= a.tol) {
                if (s.mode == kModeFp32) {
                    ns.mode = kModeFp64Redo;
                } else if (s.pending) {
                    if (PREC == kModeFp64) {
                        ns.pending = 0;
                        d.work = true;
                        d.j = s.j + 1;
                    }
                } else {
                    fin = kStatusOk;
                }
            } else if (s.j >= a.max_iter) {
                fin = kStatusNoconv;
            } else if (s.mode == PREC) {
                d.work = true;
                d.j = s.j + 1;
            }
        }
        if (d.work) {
            d.slot = s.e % 3;
            ns.e = s.e + 1;
            ns.j = d.j;
            if (PREC == kModeFp32) ns.f32 = s.f32 + 1;
        }
        if (fin >= 0) ns.status = fin;
    }
    if (stage == 0 && c.tid == 0) {
        a.st[((k + 1) & 1) * a.B + b] = ns;
        if (s.status == kActive && s.mode == kModeFp32 && (ns.mode != kModeFp32 || fin >= 0))
            atomicSub(a.ctr + 3, 1);   // leaves the FP32 phase
        if (fin >= 0) {
            a.iters[b] = s.j;
            a.rfin[2 * b] = rs;
            a.rfin[2 * b + 1] = rp;
            atomicAdd(a.ctr + 2, 1);
        }
    }
    return d;
}

template <typename T, int CX, int RY, int LX, int LY>
__device__ __forceinline__ void stage_body(const IterArgs &a, Ctx &c, int b, int i, int j, int slot)
{
    const DevProblem &P = a.P;
    constexpr int M = LX * LY;
    const int n = P.n;
    const int cur = j & 1, nxt = cur ^ 1;
    const size_t unit = (size_t)b * P.N + i;
    double *uvec = lds_ptr<double>(c, c.off.uvec);
    double *v3 = lds_ptr<double>(c, c.off.v3);
    double *kun = lds_ptr<double>(c, c.off.kun);
    double *red = lds_ptr<double>(c, c.off.red);
    unsigned long long *nrm = lds_ptr<unsigned long long>(c, c.off.nrm);

    // stage slices x_i, lam_i, x_{i-1} (x0 at i = 0), lam_{i+1} (none at
    // i = N-1), xref_i, all with the padded row stride sx = 16 * CX: a lane's
    // tile lies inside a row or entirely in its zero padding
    const bool last = (i == P.N - 1);
    const double *Xc = a.X[cur] + unit * n;
    const double *Lc = a.LAM[cur] + unit * n;
    const double *Xp = i == 0 ? a.x0 + (size_t)b * n : a.X[cur] + (unit - 1) * n;
    const double *Ln = a.LAM[cur] + (unit + 1) * n;
    const double *Xr = a.xref + (size_t)b * a.xref_inst_stride + (size_t)i * a.xref_stage_stride;
    const int ix0 = c.cl * CX, iy0 = c.G * RY;
    const int sx = 16 * CX;
    auto valid = [&](int t, int q) { return ix0 + q < P.nsx && iy0 + t < P.nsy; };
    auto pidx = [&](int t, int q) { return (iy0 + t) * sx + ix0 + q; };

    // ---- KKT rows (FP64)
    //   K^lam = lam_{i+1} - lam + h (q (x - xref) + L(k lam) + k' (L x) lam)
    //   K^x   = x_{i-1} - x + h (k L x + B u)
    const double h = P.h, kp = P.k0 * P.k1;
    StageCoef<T, CX, RY> K;
    T b1[RY][CX], b2[RY][CX];
    unsigned long long mx = 0, ml = 0;
    {
        double xc[RY][CX], lc[RY][CX], Lx[RY][CX];
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q) {
                const bool v = valid(t, q);
                xc[t][q] = v ? Xc[pidx(t, q)] : 0.0;
                lc[t][q] = v ? Lc[pidx(t, q)] : 0.0;
            }
        if (c.tid < M) uvec[c.tid] = a.U[cur][unit * M + c.tid];
        nbsum<double, CX, RY>(xc, Lx, c);
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q) Lx[t][q] -= P.c0 * xc[t][q];
        {
            double g[RY][CX], Lg[RY][CX];
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) g[t][q] = P.k0 * (1.0 + P.k1 * xc[t][q]) * lc[t][q];
            nbsum<double, CX, RY>(g, Lg, c);
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) {
                    // nodes off the grid have no KKT row: their stencil of a
                    // valid neighbour is dropped (norms, right-hand sides)
                    double kl = 0.0;
                    if (valid(t, q)) {
                        const double ln = last ? 0.0 : Ln[pidx(t, q)];
                        const double xr = Xr[pidx(t, q)];
                        const double gg = P.k0 * (1.0 + P.k1 * xc[t][q]) * lc[t][q];
                        kl = ln - lc[t][q] +
                             h * (P.q * (xc[t][q] - xr) + (Lg[t][q] - P.c0 * gg) +
                                  kp * Lx[t][q] * lc[t][q]);
                    }
                    ml = umax64(ml, abits(kl));
                    b2[t][q] = T(kl);
                }
        }
        if (c.Gv == 1) __syncthreads();   // publish uvec (no stencil barrier ran)
        {
            double Bu[RY][CX];
            b_apply<double, CX, RY, LX, LY>(uvec, c, Bu);
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) {
                    double kx = 0.0;
                    if (valid(t, q)) {
                        const double kk = P.k0 * (1.0 + P.k1 * xc[t][q]);
                        kx = Xp[pidx(t, q)] - xc[t][q] + h * (kk * Lx[t][q] + Bu[t][q]);
                    }
                    mx = umax64(mx, abits(kx));
                    b1[t][q] = T(kx);
                }
        }
        // stage coefficients of the lower layer (after the FP64 rows, so
        // their registers are not live during the residual)
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q) {
                const double kk = P.k0 * (1.0 + P.k1 * xc[t][q]);
                const double d = -1.0 - h * kk * P.c0 + h * kp * Lx[t][q];   // diag of F_x
                K.invd[t][q] = valid(t, q) ? T(1.0 / d) : T(0);
                K.cpk[t][q] = T(h * kk);
                K.g2[t][q] = T(kp * lc[t][q]);
            }
        bt_reduce<double, CX, RY, LX, LY>(lc, c, M);
    }
    unsigned long long mu = 0;
    if (c.tid < M) {
        const double ku = h * (P.r * uvec[c.tid] + red[c.tid]);   // u~ = u: no gamma term
        kun[c.tid] = ku;
        v3[c.tid] = 0.0;
        mu = abits(ku);
    }
    mx = wave_max64(mx);
    ml = wave_max64(ml);
    mu = wave_max64(mu);
    if (c.lane == 0) {
        nrm[c.w * 4 + 0] = mx;
        nrm[c.w * 4 + 1] = ml;
        nrm[c.w * 4 + 2] = mu;
    }
    __syncthreads();
    if (c.tid == 0) {
        unsigned long long ax = 0, al = 0, au = 0;
        for (int ww = 0; ww < c.W; ++ww) {
            ax = umax64(ax, nrm[ww * 4 + 0]);
            al = umax64(al, nrm[ww * 4 + 1]);
            au = umax64(au, nrm[ww * 4 + 2]);
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
        const size_t at = ((size_t)slot * a.B + b) * P.N + i;
        a.rst[at] = abits(rs);
        a.pst[at] = abits(rp);
    }
    if (a.residual_only) return;

    // ---- lower layer (T)
    const T hT = T(h), qT = T(P.q), c0T = T(P.c0);
    const double auu = h * P.r + P.gamma;
    T y5[RY][CX], y4[RY][CX];
    for (int s = 0; s < a.n_schur; ++s) {
        T cc[RY][CX];
        if (s == 0) {
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) cc[t][q] = -b1[t][q];
        } else {
            T Bv[RY][CX];
            b_apply<T, CX, RY, LX, LY>(v3, c, Bv);
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) cc[t][q] = hT * Bv[t][q] - b1[t][q];
        }
        jac_f<T, CX, RY>(cc, y5, K, a.n_sw, c);
        {
            T Ay[RY][CX];
            axx_apply<T, CX, RY>(y5, Ay, K, hT, qT, c0T, c);
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) cc[t][q] = -b2[t][q] - Ay[t][q];
        }
        jac_ft<T, CX, RY>(cc, y4, K, a.n_sw, c);
        bt_reduce<T, CX, RY, LX, LY>(y4, c, M);
        if (c.tid < M) {
            const T bt = T(red[c.tid]);
            v3[c.tid] = double((T(kun[c.tid]) + hT * bt) / T(auu));
        }
        __syncthreads();
    }
    {
        T cc[RY][CX];
        {
            T Bv[RY][CX];
            b_apply<T, CX, RY, LX, LY>(v3, c, Bv);
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) cc[t][q] = b1[t][q] - hT * Bv[t][q];
        }
        jac_f<T, CX, RY>(cc, y5, K, a.n_sw, c);          // v2 = dx
        {
            T Ay[RY][CX];
            axx_apply<T, CX, RY>(y5, Ay, K, hT, qT, c0T, c);
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) cc[t][q] = b2[t][q] - Ay[t][q];
        }
        jac_ft<T, CX, RY>(cc, y4, K, a.n_sw, c);         // v1 = dlam
    }

    // ---- update S^{j+1} = S^j - ds (FP64); x_i, lam_i re-read (L2-resident)
    double *Xn = a.X[nxt] + unit * n;
    double *Lw = a.LAM[nxt] + unit * n;
#pragma unroll
    for (int t = 0; t < RY; ++t)
#pragma unroll
        for (int q = 0; q < CX; ++q)
            if (valid(t, q)) {
                const int p = pidx(t, q);
                Xn[p] = Xc[p] - double(y5[t][q]);
                Lw[p] = Lc[p] - double(y4[t][q]);
            }
    if (c.tid < M) a.U[nxt][unit * M + c.tid] = uvec[c.tid] - v3[c.tid];
}

template <int PREC, int CX, int RY, int WB, int OCC, int LX, int LY>
__global__ void __launch_bounds__(kWave * WB, OCC) k_iterate(const IterArgs a)
{
    using T = typename std::conditional<PREC == kModeFp32, float, double>::type;
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
    c.off = lds_layout(c.GT, c.W, CX, (int)sizeof(T), LX, LY, RY);

    const int k = a.residual_only ? 0 : *(volatile const int *)(a.ctr) + a.kofs;
    // XCD-aware unit order: consecutive workgroup ids go to different XCDs, so
    // give each XCD a contiguous run of units (neighbouring stages of one
    // instance then share that XCD's L2 for the x_{i-1} / lambda_{i+1} reads).
    const int bid = blockIdx.x;
    const int unit = (bid & 7) * a.per_xcd + (bid >> 3);
    if (unit < a.units) {
        const int b = unit / a.P.N, i = unit % a.P.N;
        Decision d;
        if (a.residual_only) {
            d.work = true; d.j = 0; d.slot = a.res_slot;
        } else {
            d = decide<PREC>(a, c, b, i, k);
        }
        if (d.work) {
            double *gx = lds_ptr<double>(c, c.off.gx);
            double *gy = lds_ptr<double>(c, c.off.gy);
            float *gxf = lds_ptr<float>(c, c.off.gxf);
            float *gyf = lds_ptr<float>(c, c.off.gyf);
            for (int t = c.tid; t < LX * 16 * CX; t += blockDim.x) {
                const int aa = t / (16 * CX), ix = t % (16 * CX);
                const double v = ix < a.P.nsx ? a.gx[aa * a.P.nsx + ix] : 0.0;
                gx[t] = v;
                gxf[t] = float(v);
            }
            for (int t = c.tid; t < LY * c.GT * RY; t += blockDim.x) {
                const int bb = t / (c.GT * RY), iy = t % (c.GT * RY);
                const double v = iy < a.P.nsy ? a.gy[bb * a.P.nsy + iy] : 0.0;
                gy[t] = v;
                gyf[t] = float(v);
            }
            __syncthreads();
            stage_body<T, CX, RY, LX, LY>(a, c, b, i, d.j, d.slot);
        }
    }
}

// Consistent start from an input trajectory u (already in buffer 0): the
// states follow the backward-Euler model of eq. nlp, x_i = x_{i-1} + h f(u_i,
// x_i), solved stage by stage (K^x_i = 0), and the costates follow the
// adjoint recursion K^lam_i = 0 of Sec. 3.2 solved from i = N down to 1, i.e.
// F_x^T lam_i = -(lam_{i+1} + h q (x_i - xref_i)). Both solves are point-Jacobi
// sweeps in FP64 (for the state: on the implicit equation with k(x) taken at
// the current sweep). The costate sweeps start from the lambda already in
// buffer 0 (a supplied guess, or 0). One workgroup per instance.
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
    double *gx = lds_ptr<double>(c, c.off.gx);
    double *gy = lds_ptr<double>(c, c.off.gy);
    double *uvec = lds_ptr<double>(c, c.off.uvec);
    for (int t = c.tid; t < LX * 16 * CX; t += blockDim.x) {
        const int aa = t / (16 * CX), ix = t % (16 * CX);
        gx[t] = ix < P.nsx ? a.gx[aa * P.nsx + ix] : 0.0;
    }
    for (int t = c.tid; t < LY * c.GT * RY; t += blockDim.x) {
        const int bb = t / (c.GT * RY), iy = t % (c.GT * RY);
        gy[t] = iy < P.nsy ? a.gy[bb * P.nsy + iy] : 0.0;
    }
    const int n = P.n, sx = 16 * CX;
    const int ix0 = c.cl * CX, iy0 = c.G * RY;
    auto valid = [&](int t, int q) { return ix0 + q < P.nsx && iy0 + t < P.nsy; };
    auto pidx = [&](int t, int q) { return (iy0 + t) * sx + ix0 + q; };
    const double h = P.h, kp = P.k0 * P.k1;
    const int nsw = a.n_sw;

    // ---- states, forward in the horizon
    double xp[RY][CX];
#pragma unroll
    for (int t = 0; t < RY; ++t)
#pragma unroll
        for (int q = 0; q < CX; ++q) xp[t][q] = valid(t, q) ? a.x0[(size_t)b * n + pidx(t, q)] : 0.0;
    for (int i = 0; i < P.N; ++i) {
        const size_t unit = (size_t)b * P.N + i;
        __syncthreads();   // previous stage's readers of uvec are done
        if (c.tid < M) uvec[c.tid] = a.U[0][unit * M + c.tid];
        __syncthreads();
        double Bu[RY][CX], x[RY][CX];
        b_apply<double, CX, RY, LX, LY>(uvec, c, Bu);
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q) x[t][q] = xp[t][q];
        for (int s = 0; s < nsw; ++s) {
            double nb[RY][CX];
            nbsum<double, CX, RY>(x, nb, c);
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) {
                    const double kk = P.k0 * (1.0 + P.k1 * x[t][q]);
                    const double v = (xp[t][q] + h * kk * nb[t][q] + h * Bu[t][q]) /
                                     (1.0 + h * kk * P.c0);
                    x[t][q] = valid(t, q) ? v : 0.0;
                }
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
        double x[RY][CX], Lx[RY][CX], lam[RY][CX];
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q) {
                x[t][q] = valid(t, q) ? Xi[pidx(t, q)] : 0.0;
                lam[t][q] = valid(t, q) ? Li[pidx(t, q)] : 0.0;
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
        for (int s = 0; s < nsw; ++s) {
            double z[RY][CX], nb[RY][CX];
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) z[t][q] = cpk[t][q] * lam[t][q];
            nbsum<double, CX, RY>(z, nb, c);
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) lam[t][q] = (cc[t][q] - nb[t][q]) * invd[t][q];
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
// 1 (slot 1). start_used[b] = used_if_kept, or 0 (the buffer-1 start).
__global__ void k_choose_flags(const IterArgs a, int *start_used, int used_if_kept)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.units) return;
    const size_t N = a.P.N;
    unsigned long long mw = 0, mc = 0;
    for (size_t i = 0; i < N; ++i) {
        mw = umax64(mw, a.rst[(size_t)b * N + i]);
        mc = umax64(mc, a.rst[((size_t)a.B + b) * N + i]);
    }
    start_used[b] = (bits2d(mw) <= bits2d(mc)) ? used_if_kept : 0;
}

// Copy buffer 1's start over buffer 0 for the instances that fell back.
__global__ void k_choose_copy(const IterArgs a, const int *start_used)
{
    const size_t np = a.P.n, N = a.P.N, m = a.P.m;
    const size_t per = N * (2 * np + m);
    const size_t tot = (size_t)a.units * per, stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
        const size_t b = t / per, r = t % per;
        if (start_used[b] != 0) continue;
        if (r < N * np) {
            a.X[0][b * N * np + r] = a.X[1][b * N * np + r];
        } else if (r < 2 * N * np) {
            const size_t q = r - N * np;
            a.LAM[0][b * N * np + q] = a.LAM[1][b * N * np + q];
        } else {
            const size_t q = r - 2 * N * np;
            a.U[0][b * N * m + q] = a.U[1][b * N * m + q];
        }
    }
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
    const size_t nN = (size_t)a.count * a.N * np;
    const size_t mN = (size_t)a.count * a.N * a.m;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < nN; t += stride) {
        const size_t unit = t / np, p = t % np;
        const int row = (int)(p / a.sx), col = (int)(p % a.sx);
        const size_t b = unit / a.N;
        double x = 0.0, l = 0.0;
        if (col < a.nsx) {
            const size_t dense = unit * (size_t)a.nsx * a.nsy + (size_t)row * a.nsx + col;
            x = a.wx ? a.wx[dense] : a.x0[b * np + p];
            l = a.wl ? a.wl[dense] : 0.0;
        }
        a.X[t] = x;
        a.LAM[t] = l;
    }
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < mN; t += stride)
        a.U[t] = a.wu ? a.wu[t] : 0.0;
    if (a.trajectory_only) return;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)a.count;
         t += stride) {
        InstState s;
        s.status = kActive; s.mode = a.mode; s.e = 0; s.j = 0; s.pending = 0; s.f32 = 0;
        s.pad[0] = s.pad[1] = 0;
        a.st[t] = s;
        a.st[a.B + t] = s;
        a.iters[t] = 0;
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

// Copy each instance's returned iterate (buffer iters[b] & 1) out, from the
// padded stage layout to the dense [count][N][n] layout.
__global__ void k_output(const OutArgs a)
{
    const size_t n = (size_t)a.nsx * a.nsy, np = (size_t)a.nsy * a.sx;
    const size_t w = (size_t)a.N * n, wm = (size_t)a.N * a.m;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)a.count * w;
         t += stride) {
        const size_t unit = t / n, p = t % n;
        const int b = (int)(t / w);
        const int buf = a.iters[b] & 1;
        const size_t src = unit * np + (p / a.nsx) * a.sx + p % a.nsx;
        a.ox[t] = a.X[buf][src];
        a.ol[t] = a.LAM[buf][src];
    }
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)a.count * wm;
         t += stride) {
        const int b = (int)(t / wm);
        a.ou[t] = a.U[a.iters[b] & 1][t];
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
    NMPC_TILE(kModeFp32, 6, 2, 12)                                                  \
    NMPC_TILE(kModeFp64, 1, 4, 4) NMPC_TILE(kModeFp64, 2, 2, 8)                     \
    NMPC_TILE(kModeFp64, 2, 4, 4) NMPC_TILE(kModeFp64, 3, 2, 8)                     \
    NMPC_TILE(kModeFp64, 4, 2, 8)                                                   \
    NMPC_TILE(kModeFp64, 6, 2, 12)

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
    NMPC_ROLL(6, 2, 12)

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
const void *choose_flags_kernel() { return (const void *)&k_choose_flags; }
const void *choose_copy_kernel() { return (const void *)&k_choose_copy; }
const void *pad_kernel() { return (const void *)&k_pad; }
const void *advance_kernel() { return (const void *)&k_advance; }
const void *output_kernel() { return (const void *)&k_output; }

}  // namespace nmpc
