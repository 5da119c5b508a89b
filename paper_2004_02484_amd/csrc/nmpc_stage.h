// nmpc_stage.h -- device code of one (instance, stage) unit of the upper
// iteration, shared by the batch kernel (one problem per launch) and the
// ragged kernel (instances of several grids and horizons in one launch).
//
// The stage grid is held in registers as tiles: 16 lanes span a grid row,
// each lane owning CX consecutive columns and RY consecutive rows; the four
// 16-lane rows of a wave and the waves of the workgroup stack downwards.
// Stencil neighbours inside a tile are registers, the left/right tile edges
// come from the adjacent lane by DPP row shifts (VALU, zero-filled at the row
// ends, which is the Dirichlet value), and only the top/bottom tile rows pass
// through LDS.
#pragma once

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

// Edge slots of the tile-row exchange: two regions (alternating by flip, so a
// wave that is still reading one exchange's edges is never overwritten by the
// next exchange), each holding the top and the bottom tile rows of every lane
// in 8-byte slots. The region offset is in bytes, the same for every value
// type, so exchanges of double and float values may follow each other.
template <typename V, int CX>
__device__ __forceinline__ V *edge_region(const Ctx &c)
{
    return reinterpret_cast<V *>(c.lds + c.off.edge + (size_t)c.flip * 2 * c.GT * 16 * CX * 8);
}

// o = N(v) from the tile and the rows above / below it.
template <typename V, int CX, int RY>
__device__ __forceinline__ void stencil(const V (&v)[RY][CX], const V (&above)[CX],
                                        const V (&below)[CX], V (&o)[RY][CX], const Ctx &c)
{
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

// Neighbour sum N(v)_p = (v_l + v_r)/dx^2 + (v_u + v_d)/dy^2 with zero values
// off the grid (the Laplacian is L v = N(v) - (2/dx^2 + 2/dy^2) v).
template <typename V, int CX, int RY>
__device__ __forceinline__ void nbsum(const V (&v)[RY][CX], V (&o)[RY][CX], Ctx &c)
{
    V above[CX], below[CX];
#pragma unroll
    for (int q = 0; q < CX; ++q) { above[q] = V(0); below[q] = V(0); }
    if (c.Gv > 1) {   // tile rows shared through LDS
        V *top = edge_region<V, CX>(c);
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
    stencil<V, CX, RY>(v, above, below, o, c);
}

// N(v1) and N(v2) with one exchange: for float tiles both arrays' edge values
// share a slot, so one barrier serves both; double tiles take two exchanges.
template <typename V, int CX, int RY>
__device__ __forceinline__ void nbsum2(const V (&v1)[RY][CX], const V (&v2)[RY][CX],
                                       V (&o1)[RY][CX], V (&o2)[RY][CX], Ctx &c)
{
    if constexpr (sizeof(V) != 4) {
        nbsum<V, CX, RY>(v1, o1, c);
        nbsum<V, CX, RY>(v2, o2, c);
    } else {
        float a1[CX], b1[CX], a2[CX], b2[CX];
#pragma unroll
        for (int q = 0; q < CX; ++q) { a1[q] = 0.f; b1[q] = 0.f; a2[q] = 0.f; b2[q] = 0.f; }
        if (c.Gv > 1) {
            float2 *top = edge_region<float2, CX>(c);
            float2 *bot = top + (size_t)c.GT * 16 * CX;
            const int me = (c.G * 16 + c.cl) * CX;
#pragma unroll
            for (int q = 0; q < CX; ++q) {
                top[me + q] = make_float2(v1[0][q], v2[0][q]);
                bot[me + q] = make_float2(v1[RY - 1][q], v2[RY - 1][q]);
            }
            __syncthreads();
            if (c.G > 0) {
#pragma unroll
                for (int q = 0; q < CX; ++q) {
                    const float2 e = bot[me - 16 * CX + q];
                    a1[q] = e.x;
                    a2[q] = e.y;
                }
            }
            if (c.G + 1 < c.Gv) {
#pragma unroll
                for (int q = 0; q < CX; ++q) {
                    const float2 e = top[me + 16 * CX + q];
                    b1[q] = e.x;
                    b2[q] = e.y;
                }
            }
            c.flip ^= 1;
        }
        stencil<float, CX, RY>(v1, a1, b1, o1, c);
        stencil<float, CX, RY>(v2, a2, b2, o2, c);
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

// (B^T y)_j for j < M, left in red[j] (double) by thread j, which is the only
// thread that reads it before the next barrier (with one tile row, where the
// stencils take no barrier, all threads are synchronized on return). Per lane: column partials t_b = sum_t gy[b][iy_t] y_t, then the
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
    if (c.Gv == 1) __syncthreads();
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
    T nb1[RY][CX], nb2[RY][CX], z[RY][CX];
#pragma unroll
    for (int t = 0; t < RY; ++t)
#pragma unroll
        for (int p = 0; p < CX; ++p) z[t][p] = K.g2[t][p] * y[t][p];
    nbsum2<T, CX, RY>(y, z, nb1, nb2, c);
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
//   REDO (FP64 kernel)             -> re-evaluate S^j in FP64: its update is the
//                                     FP64 step S^{j+1}; owe the evaluation of S^{j+1}
//   FP64 mode, test passed, owed   -> evaluate S^{j+1} (its own test decides)
//   FP64 mode, test passed         -> finished, S^j returned
// Nb: the instance's stages; rbase: offset of its stage residuals within a
// residual slot (slot stride a.rslot).
template <int PREC>
__device__ Decision decide(const IterArgs &a, Ctx &c, int b, int stage, int k, int Nb,
                           long long rbase)
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
            const size_t base = (size_t)((s.e - 1) % 3) * a.rslot + rbase;
            unsigned long long ms = 0, mp = 0;
            for (int t = c.lane; t < Nb; t += kWave) {
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

// Where one unit's data lives: its instance's trajectories start at element
// so (X, LAM) and uo (U) of the iterate buffers, its padded x0 at xo and its
// xref_i at xro; i is the stage. The stage reads s_i from buffer src and
// writes its new value to buffer dst; the neighbour values x_{i-1} and
// lambda_{i+1} that enter the update come from buffers xpb / lnb, those that
// enter the residual of S^j from xrb / lrb (they differ in Gauss-Seidel
// sweeps, where the update sees neighbours already updated in this sweep).
// utb >= 0 names the buffer of the regularization reference u~ when it is not
// the stage's own input (then K^u carries gamma (u - u~)). The pointers
// themselves stay in the kernel arguments, which the compiler may reload
// instead of keeping them live.
struct StageLoc {
    long long so, uo, xo, xro;
    long long res_at;              // >= 0: index into a.rst / a.pst; -1: accumulate into
                                   // the caller's norms only; -2: no residual
    int i, src, dst, xpb, xrb, lnb, lrb, utb;
    bool last;                     // i is the last stage
    bool res_only;                 // stop after the residual (no lower layer, no update)
    bool pf;                       // x_i, lambda_i are in the LDS prefetch region
    int pnb, pni;                  // stage pni of buffer pnb is prefetched once this stage
                                   // has read its own (pnb < 0: none)
};

// Start the copy of x and lambda (n doubles each, padded layout) into the LDS
// prefetch region at c.off.total: global -> LDS transfers of 16 bytes per lane,
// 1 KB per wave instruction, spread over the waves. They complete in the
// background; the data may be read after s_waitcnt and a barrier. Lanes past
// the end re-read the last 16 bytes into slots nobody reads (n is even).
__device__ __forceinline__ void prefetch_xl(const Ctx &c, const double *x, const double *l, int n)
{
    typedef const __attribute__((address_space(1))) void *GPtr;
    typedef __attribute__((address_space(3))) void *LPtr;
    const int chunks = (n * 8 + 1023) / 1024;
    const int npf = chunks * 128;
    double *base = lds_ptr<double>(c, c.off.total);
    for (int ch = c.w; ch < 2 * chunks; ch += c.W) {
        const bool isl = ch >= chunks;
        const int cc = isl ? ch - chunks : ch;
        int e = cc * 128 + c.lane * 2;
        e = e < n - 2 ? e : n - 2;
        const double *src = (isl ? l : x) + e;
        double *dst = base + (isl ? npf : 0) + cc * 128;
        __builtin_amdgcn_global_load_lds((GPtr)src, (LPtr)dst, 16, 0, 0);
    }
}

__device__ __forceinline__ StageLoc jacobi_loc(int cur)
{
    StageLoc v{};
    v.src = v.xpb = v.xrb = v.lnb = v.lrb = cur;
    v.dst = cur ^ 1;
    v.utb = -1;
    v.pnb = -1;
    return v;
}

// 1 / d for the lower layer's diagonal: the FP32 kernels use the hardware
// reciprocal (about 1 ulp; the coefficient only shapes the preconditioner,
// the FP64 residual decides), the FP64 kernels the correctly rounded quotient.
template <typename T>
__device__ __forceinline__ T recip(double d);
template <>
__device__ __forceinline__ float recip<float>(double d) { return __builtin_amdgcn_rcpf(float(d)); }
template <>
__device__ __forceinline__ double recip<double>(double d) { return 1.0 / d; }

// acc (thread 0 only): running bit-pattern max of (r_scaled, r_paper) over
// the stages processed with res_at == -1.
template <typename T, int CX, int RY, int LX, int LY>
__device__ __forceinline__ void stage_body(const IterArgs &a, const DevProblem &P,
                                           const StageLoc &v, Ctx &c,
                                           unsigned long long (&acc)[2])
{
    constexpr int M = LX * LY;
    const int n = P.n;
    double *uvec = lds_ptr<double>(c, c.off.uvec);
    double *v3 = lds_ptr<double>(c, c.off.v3);
    double *kun = lds_ptr<double>(c, c.off.kun);
    double *red = lds_ptr<double>(c, c.off.red);
    unsigned long long *nrm = lds_ptr<unsigned long long>(c, c.off.nrm);

    const StageLoc &sv = v;
    // stage slices x_i, lam_i, x_{i-1} (x0 at i = 0), lam_{i+1} (none at the
    // last stage), xref_i, all with the padded row stride sx = 16 * CX: a
    // lane's tile lies inside a row or entirely in its zero padding
    const bool last = v.last;
    const bool want_res = v.res_at != -2;
    const size_t si = (size_t)v.so + (size_t)v.i * n;
    const double *Xc = a.X[v.src] + si;
    const double *Lc = a.LAM[v.src] + si;
    const double *Xp = v.i == 0 ? a.x0 + v.xo : a.X[v.xpb] + (si - n);
    const double *Xq = v.i == 0 ? Xp : a.X[v.xrb] + (si - n);
    const double *Ln = a.LAM[v.lnb] + (si + n);
    const double *Lq = a.LAM[v.lrb] + (si + n);
    const bool xdiff = want_res && v.i > 0 && v.xrb != v.xpb;
    const bool ldiff = want_res && !last && v.lrb != v.lnb;
    const double *Xr = a.xref + v.xro;
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
                if (sv.pf) {
                    const double *px = lds_ptr<double>(c, c.off.total);
                    xc[t][q] = v ? px[pidx(t, q)] : 0.0;
                    lc[t][q] = v ? px[gs_pf_doubles(n) + pidx(t, q)] : 0.0;
                } else {
                    xc[t][q] = v ? Xc[pidx(t, q)] : 0.0;
                    lc[t][q] = v ? Lc[pidx(t, q)] : 0.0;
                }
            }
        if (c.tid < M) uvec[c.tid] = a.U[v.src][v.uo + (size_t)v.i * M + c.tid];
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
                    double kl = 0.0, klr = 0.0;
                    if (valid(t, q)) {
                        const double ln = last ? 0.0 : Ln[pidx(t, q)];
                        const double xr = Xr[pidx(t, q)];
                        const double gg = P.k0 * (1.0 + P.k1 * xc[t][q]) * lc[t][q];
                        const double rest = h * (P.q * (xc[t][q] - xr) + (Lg[t][q] - P.c0 * gg) +
                                                 kp * Lx[t][q] * lc[t][q]);
                        kl = ln - lc[t][q] + rest;
                        klr = ldiff ? Lq[pidx(t, q)] - lc[t][q] + rest : kl;
                    }
                    ml = umax64(ml, abits(klr));
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
                    double kx = 0.0, kxr = 0.0;
                    if (valid(t, q)) {
                        const double kk = P.k0 * (1.0 + P.k1 * xc[t][q]);
                        const double fx = h * (kk * Lx[t][q] + Bu[t][q]);
                        kx = Xp[pidx(t, q)] - xc[t][q] + fx;
                        kxr = xdiff ? Xq[pidx(t, q)] - xc[t][q] + fx : kx;
                    }
                    mx = umax64(mx, abits(kxr));
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
                K.invd[t][q] = valid(t, q) ? recip<T>(d) : T(0);
                K.cpk[t][q] = T(h * kk);
                K.g2[t][q] = T(kp * lc[t][q]);
            }
        bt_reduce<double, CX, RY, LX, LY>(lc, c, M);
    }
    unsigned long long mu = 0;
    if (c.tid < M) {
        // with u~ = u^k the gamma term vanishes at evaluation; a stage whose
        // reference is another buffer's input (second sweep of SGS) keeps it
        const double ku = h * (P.r * uvec[c.tid] + red[c.tid]);
        const double reg = v.utb >= 0
            ? P.gamma * (uvec[c.tid] - a.U[v.utb][v.uo + (size_t)v.i * M + c.tid]) : 0.0;
        kun[c.tid] = ku + reg;
        v3[c.tid] = 0.0;
        mu = abits(ku);
    }
    if (want_res) {
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
            if (v.res_at >= 0) {
                a.rst[v.res_at] = abits(rs);
                a.pst[v.res_at] = abits(rp);
            } else {
                acc[0] = umax64(acc[0], abits(rs));
                acc[1] = umax64(acc[1], abits(rp));
            }
        }
    } else {
        __syncthreads();   // publish kun / v3 (the norm path's barrier)
    }
    // every wave has read its x_i, lambda_i (before the first stencil barrier):
    // the prefetch region may take the next stage's
    if (v.pnb >= 0) {
        const size_t sn = (size_t)v.so + (size_t)v.pni * n;
        prefetch_xl(c, a.X[v.pnb] + sn, a.LAM[v.pnb] + sn, n);
    }
    if (a.residual_only || v.res_only) return;

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
    double *Xn = a.X[v.dst] + si;
    double *Lw = a.LAM[v.dst] + si;
#pragma unroll
    for (int t = 0; t < RY; ++t)
#pragma unroll
        for (int q = 0; q < CX; ++q)
            if (valid(t, q)) {
                const int p = pidx(t, q);
                Xn[p] = Xc[p] - double(y5[t][q]);
                Lw[p] = Lc[p] - double(y4[t][q]);
            }
    if (c.tid < M) a.U[v.dst][v.uo + (size_t)v.i * M + c.tid] = uvec[c.tid] - v3[c.tid];
}

// The separable input factors gx [LX][nsx], gy [LY][nsy] into LDS (double and
// float copies), laid out for the tile: gx by padded column, gy by tile row.
template <int CX, int RY, int LX, int LY>
__device__ __forceinline__ void load_tables(Ctx &c, const double *gxs, const double *gys, int nsx,
                                            int nsy)
{
    double *gx = lds_ptr<double>(c, c.off.gx);
    double *gy = lds_ptr<double>(c, c.off.gy);
    float *gxf = lds_ptr<float>(c, c.off.gxf);
    float *gyf = lds_ptr<float>(c, c.off.gyf);
    for (int t = c.tid; t < LX * 16 * CX; t += c.W * kWave) {
        const int aa = t / (16 * CX), ix = t % (16 * CX);
        const double v = ix < nsx ? gxs[aa * nsx + ix] : 0.0;
        gx[t] = v;
        gxf[t] = float(v);
    }
    for (int t = c.tid; t < LY * c.GT * RY; t += c.W * kWave) {
        const int bb = t / (c.GT * RY), iy = t % (c.GT * RY);
        const double v = iy < nsy ? gys[bb * nsy + iy] : 0.0;
        gy[t] = v;
        gyf[t] = float(v);
    }
    __syncthreads();
}

// Workgroup geometry for a CX x RY tile on a grid of nsy rows.
template <typename T, int CX, int RY, int LX, int LY>
__device__ __forceinline__ void tile_setup(Ctx &c, const DevProblem &P)
{
    c.tid = threadIdx.x;
    c.lane = c.tid & (kWave - 1);
    c.cl = c.lane & 15;
    c.w = c.tid / kWave;
    c.W = blockDim.x / kWave;
    c.G = c.w * 4 + (c.lane >> 4);
    c.GT = c.W * 4;
    c.Gv = (P.nsy + RY - 1) / RY;
    c.flip = 0;
    c.ax = P.idx2;
    c.ay = P.idy2;
    c.off = lds_layout(c.GT, c.W, CX, (int)sizeof(T), LX, LY, RY);
}

}  // namespace nmpc
