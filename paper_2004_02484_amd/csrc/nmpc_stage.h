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
// type, so exchanges of double and float values may follow each other. Slots
// are column-major within a tile row set: value q of lane-row G, lane cl sits
// at q * 16 GT + 16 G + cl, so the 64 lanes of a wave touch consecutive slots
// (no LDS bank conflicts).
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
        const int me = c.G * 16 + c.cl, qs = c.GT * 16;
#pragma unroll
        for (int q = 0; q < CX; ++q) { top[q * qs + me] = v[0][q]; bot[q * qs + me] = v[RY - 1][q]; }
        __syncthreads();
        if (c.G > 0) {
#pragma unroll
            for (int q = 0; q < CX; ++q) above[q] = bot[q * qs + me - 16];
        }
        if (c.G + 1 < c.Gv) {
#pragma unroll
            for (int q = 0; q < CX; ++q) below[q] = top[q * qs + me + 16];
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
            const int me = c.G * 16 + c.cl, qs = c.GT * 16;
#pragma unroll
            for (int q = 0; q < CX; ++q) {
                top[q * qs + me] = make_float2(v1[0][q], v2[0][q]);
                bot[q * qs + me] = make_float2(v1[RY - 1][q], v2[RY - 1][q]);
            }
            __syncthreads();
            if (c.G > 0) {
#pragma unroll
                for (int q = 0; q < CX; ++q) {
                    const float2 e = bot[q * qs + me - 16];
                    a1[q] = e.x;
                    a2[q] = e.y;
                }
            }
            if (c.G + 1 < c.Gv) {
#pragma unroll
                for (int q = 0; q < CX; ++q) {
                    const float2 e = top[q * qs + me + 16];
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

// Lane exchanges on the VALU, without LDS instructions: xpart<MASK>(v) is the
// value of lane l ^ MASK. Masks 32 and 16 use the gfx950 half-swaps
// (v_permlane32_swap: lanes 32..63 of the first operand trade places with
// lanes 0..31 of the second; v_permlane16_swap: the odd 16-lane rows of the
// first with the even rows of the second); masks 8, 2, 1 are DPP row / quad
// permutations, mask 4 a pair of DPP row shifts.
template <int MASK>
__device__ __forceinline__ unsigned xpart_u32(unsigned v, int lane)
{
    if constexpr (MASK == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? r[0] : r[1];
    } else if constexpr (MASK == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? r[0] : r[1];
    } else if constexpr (MASK == 8) {
        return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);   // row_ror:8
    } else if constexpr (MASK == 4) {
        const int dn = __builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);   // row_shr:4
        const int up = __builtin_amdgcn_update_dpp(0, (int)v, 0x104, 0xF, 0xF, true);   // row_shl:4
        return (unsigned)((lane & 4) ? dn : up);
    } else if constexpr (MASK == 2) {
        return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad 2,3,0,1
    } else {
        static_assert(MASK == 1, "xor masks 32 .. 1");
        return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad 1,0,3,2
    }
}

template <int MASK>
__device__ __forceinline__ float xpart(float v, int lane)
{
    return __uint_as_float(xpart_u32<MASK>(__float_as_uint(v), lane));
}
template <int MASK>
__device__ __forceinline__ unsigned long long xpart(unsigned long long v, int lane)
{
    const unsigned lo = xpart_u32<MASK>((unsigned)v, lane);
    const unsigned hi = xpart_u32<MASK>((unsigned)(v >> 32), lane);
    return ((unsigned long long)hi << 32) | lo;
}
template <int MASK>
__device__ __forceinline__ double xpart(double v, int lane)
{
    return __longlong_as_double((long long)xpart<MASK>((unsigned long long)__double_as_longlong(v), lane));
}

// One reduce-scatter step of mask MASK: lanes without the mask bit keep x
// summed with their partner's x, lanes with it keep y summed with their
// partner's y. For masks 32 and 16 the two outputs of the half-swap of (x, y)
// are exactly these pairs, so no selection is needed.
template <int MASK, typename V>
__device__ __forceinline__ V rs_pair(V x, V y, int lane)
{
    if constexpr (MASK == 32 || MASK == 16) {
        V r0, r1;
        if constexpr (sizeof(V) == 4) {
            const unsigned bx = __float_as_uint(x), by = __float_as_uint(y);
            const auto r = MASK == 32 ? __builtin_amdgcn_permlane32_swap(bx, by, false, false)
                                      : __builtin_amdgcn_permlane16_swap(bx, by, false, false);
            r0 = __uint_as_float(r[0]);
            r1 = __uint_as_float(r[1]);
        } else {
            const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
            const unsigned xl = (unsigned)bx, xh = (unsigned)(bx >> 32);
            const unsigned yl = (unsigned)by, yh = (unsigned)(by >> 32);
            const auto lo = MASK == 32 ? __builtin_amdgcn_permlane32_swap(xl, yl, false, false)
                                       : __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
            const auto hi = MASK == 32 ? __builtin_amdgcn_permlane32_swap(xh, yh, false, false)
                                       : __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
            r0 = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
            r1 = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
        }
        return r0 + r1;
    } else {
        const bool up = (lane & MASK) != 0;
        const V send = up ? x : y, keep = up ? y : x;
        return keep + xpart<MASK>(send, lane);
    }
}

// Sum over the lanes that differ only in the bits MASK, MASK / 2, ..., 1.
template <int MASK, typename V>
__device__ __forceinline__ V allreduce_from(V s, int lane)
{
    if constexpr (MASK >= 1) {
        s += xpart<MASK>(s, lane);
        return allreduce_from<MASK / 2>(s, lane);
    } else {
        return s;
    }
}

// Reduce-scatter of MP per-lane values over the 64 lanes, the halving steps
// taking masks MASK, MASK / 2, ... and the rest full butterflies: on return
// lane l holds the wave total of the element whose index is made of l's bits
// at the halving masks (l >> (log2(MASK) + 1 - log2(MP)) for the lanes
// below 2 MASK). Each halving step trades the half a lane does not keep with
// its partner, so the exchange volume is about the element count instead of
// 6x it.
template <int MP, int MASK, typename V>
__device__ __forceinline__ V reduce_scatter(V (&a)[MP], int lane)
{
    if constexpr (MP == 1) {
        return allreduce_from<MASK>(a[0], lane);
    } else {
        constexpr int HALF = MP / 2;
        V b[HALF];
#pragma unroll
        for (int j = 0; j < HALF; ++j) b[j] = rs_pair<MASK>(a[j], a[j + HALF], lane);
        return reduce_scatter<HALF, MASK / 2>(b, lane);
    }
}

template <int MASK = 32>
__device__ __forceinline__ unsigned long long wave_max64(unsigned long long v, int lane)
{
    if constexpr (MASK >= 1) {
        v = umax64(v, xpart<MASK>(v, lane));
        return wave_max64<MASK / 2>(v, lane);
    } else {
        return v;
    }
}

// (B v)_p = sum_b gy[b][iy] sum_a gx[a][ix] v[b*LX + a]; v in LDS (double).
// The gx table holds gx[a][cl * CX + q] at (a * CX + q) * 16 + cl, so the 16
// lanes of a tile row read consecutive values.
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
                acc += V(gx[(a * CX + q) * 16 + c.cl]) * V(vs[b * LX + a]);
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

// (B^T y)_j for j < M, returned to lane j of every wave (each wave sums the
// waves' partials itself, in wave order, so all waves hold the same values).
// The partials stay in LDS until the next barrier; with one tile row, where
// the stencils take no barrier, all threads are synchronized on return. Per
// lane: column partials t_b = sum_t gy[b][iy_t] y_t, then the products with
// gx are formed inside the first halving step of the cross-lane reduction,
// then the waves' partials are summed.
template <typename V, int CX, int RY, int LX, int LY>
__device__ __forceinline__ V bt_reduce(const V (&y)[RY][CX], Ctx &c, int M)
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
            for (int q = 0; q < CX; ++q) acc += V(gx[((j % LX) * CX + q) * 16 + c.cl]) * tb[j / LX][q];
        }
        return acc;
    };
    V e;
    if constexpr (MP == 1) {
        e = allreduce_from<32>(prod(0), c.lane);
    } else {
        constexpr int HALF = MP / 2;
        V a[HALF];
#pragma unroll
        for (int j = 0; j < HALF; ++j) a[j] = rs_pair<32>(prod(j), prod(j + HALF), c.lane);
        e = reduce_scatter<HALF, 16>(a, c.lane);
    }
    constexpr int SH = 6 - Pow2<MP>::lg;
    if ((c.lane & ((1 << SH) - 1)) == 0) red[c.w * kMaxM + (c.lane >> SH)] = double(e);
    __syncthreads();
    V s = V(0);
    if (c.lane < M)
        for (int ww = 0; ww < c.W; ++ww) s += V(red[ww * kMaxM + c.lane]);
    if (c.Gv == 1) __syncthreads();
    return s;
}

// The M values v (lane j of the wave holds element j) to every lane, as
// wave-uniform values (v_readlane into scalar registers).
template <typename T, int M>
__device__ __forceinline__ void wave_bcast(double v, T (&o)[M])
{
    if constexpr (sizeof(T) == 4) {
        const int b = __float_as_int(float(v));
#pragma unroll
        for (int j = 0; j < M; ++j) o[j] = __int_as_float(__builtin_amdgcn_readlane(b, j));
    } else {
        const long long b = __double_as_longlong(v);
        const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const unsigned l = (unsigned)__builtin_amdgcn_readlane(lo, j);
            const unsigned hh = (unsigned)__builtin_amdgcn_readlane(hi, j);
            o[j] = T(__longlong_as_double((long long)(((unsigned long long)hh << 32) | l)));
        }
    }
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
    bool work;       // evaluate (and update) in this kernel
    int j;           // index of the iterate evaluated (S^j)
    int slot;        // residual slot this evaluation accumulates into
    bool eval_only;  // evaluate S^j only: its test is the last one owed
    bool redo;       // the FP64 correction step from the FP32-sweep iterate S^j
};

// Per-instance state machine. All workgroups of an instance compute the same
// decision from data that no one writes during this kernel (the state slot of
// this kernel's parity and the per-stage residuals of the instance's previous
// evaluation, max-reduced here); the stage-0 workgroup publishes the next
// state into the other parity slot. PREC is this kernel's precision (kModeFp32 or kModeFp64); an
// instance in another mode waits for the kernel of its precision.
//   FP32 mode, test passed at S^j  -> REDO (FP32-active count decremented),
//                                     or finished with S^j when a.fp32_finish
//   REDO (FP64 kernel)             -> re-evaluate S^j in FP64: its update is the
//                                     FP64 step S^{j+1}; owe the evaluation of S^{j+1}
//   FP64 mode, test passed, owed   -> evaluate S^{j+1} without an update (its
//                                     own test decides; a failed test makes
//                                     the next step re-evaluate S^{j+1}); the
//                                     FP32 kernel takes this too in a launch
//                                     with a.eval_fp64
//   FP64 mode, test passed         -> finished, S^j returned
// Nb: the instance's stages; rbase: offset of its stage residuals within a
// residual slot (slot stride a.rslot).
template <int PREC>
__device__ Decision decide(const IterArgs &a, Ctx &c, int b, int stage, int k, int Nb,
                           long long rbase)
{
    // up to 64 stages: the stage norms of all three residual slots are
    // requested together with the state, so the decision waits for memory once
    const bool one_row = Nb <= kWave;
    unsigned long long r3[3] = {0, 0, 0}, p3[3] = {0, 0, 0};
    if (one_row && c.lane < Nb) {
#pragma unroll
        for (int sl = 0; sl < 3; ++sl) {
            r3[sl] = a.rst[(size_t)sl * a.rslot + rbase + c.lane];
            p3[sl] = a.pst[(size_t)sl * a.rslot + rbase + c.lane];
        }
    }
    const InstState s = a.st[(k & 1) * a.B + b];
    InstState ns = s;
    Decision d{false, 0, 0, false, false};
    int fin = -1;
    double rs = 0.0, rp = 0.0;
    if (s.status == kActive && s.e > 0) {
        // max over the stages' residuals of the previous evaluation, taken by
        // every wave itself (no LDS and no barrier); NaN bit patterns order
        // above every finite value
        const int sl = (s.e - 1) % 3;
        unsigned long long ms = 0, mp = 0;
        if (one_row) {
            ms = sl == 0 ? r3[0] : sl == 1 ? r3[1] : r3[2];
            mp = sl == 0 ? p3[0] : sl == 1 ? p3[1] : p3[2];
        } else {
            const size_t base = (size_t)sl * a.rslot + rbase;
            for (int t = c.lane; t < Nb; t += kWave) {
                ms = umax64(ms, a.rst[base + t]);
                mp = umax64(mp, a.pst[base + t]);
            }
        }
        rs = bits2d(wave_max64(ms, c.lane));
        rp = bits2d(wave_max64(mp, c.lane));
    }
    const double rt = a.res_paper ? rp : rs;   // the norm the test is on
    if (s.status == kActive) {
        if (s.e == 0) {
            if (s.mode == PREC) { d.work = true; d.j = 0; }
        } else {
            if (!(rt <= 1.7976931348623157e308)) {            // NaN or Inf
                fin = kStatusNonfinite;
            } else if (s.mode == kModeFp64Redo) {
                if (PREC == kModeFp64) {
                    ns.mode = kModeFp64;
                    ns.pending = 1;
                    d.work = true;
                    d.j = s.j;
                    d.redo = true;
                }
            } else if (rt <= a.tol) {
                if (s.mode == kModeFp32) {
                    if (a.fp32_finish) fin = kStatusOk;
                    else ns.mode = kModeFp64Redo;
                } else if (s.pending) {
                    // an evaluation only: the FP32 kernel may take it when
                    // the launch asks (its residual is the same FP64 code)
                    if (PREC == kModeFp64 || a.eval_fp64) {
                        ns.pending = 0;
                        d.work = true;
                        d.j = s.j + 1;
                        d.eval_only = true;
                    }
                } else {
                    fin = kStatusOk;
                }
            } else if (s.j >= a.max_iter) {
                fin = kStatusNoconv;
            } else if (s.mode == PREC) {
                d.work = true;
                d.j = s.eonly ? s.j : s.j + 1;   // no S^{j+1} after an evaluation-only kernel
            }
        }
        if (d.work) {
            d.slot = s.e % 3;
            ns.e = s.e + 1;
            ns.j = d.j;
            ns.eonly = d.eval_only ? 1 : 0;
            if (PREC == kModeFp32 && s.mode == kModeFp32) ns.f32 = s.f32 + 1;
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
    double omega;                  // the update is S^j - omega ds (1: the plain step)
    long long box_at;              // >= 0: index into a.apart for this stage's step limit
    long long du_at;               // >= 0: instance whose FP64 correction step this is
                                   // (max |du|, max |u_new| into a.du)
    const double *tgx, *tgy;       // non-null: load the input tables after issuing the
                                   // stage's loads (their first reader follows a barrier)
    bool xp_lds;                   // copy x_{i-1} into LDS at the start, then x_i for the
                                   // update during the lower layer (a.xp_lds)
    bool defer_norms;              // one stage per workgroup: combine the waves' norm
                                   // partials after the lower layer's first barrier
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

// Start the copy of one array of n doubles (padded layout) into LDS at
// c.off.total, 16 bytes per lane (1 KB per wave instruction) spread over the
// waves, without registers; read after s_waitcnt and a barrier. Lanes past the
// end re-read the last 16 bytes into slots nobody reads (n is even).
// A lane's tile of a padded stage slice (row stride 16 CX): rows past the
// grid are not read; columns past the grid read the row's padding, which is
// masked to zero here, so the even-width tiles load 16 bytes at a time.
template <int CX, int RY>
__device__ __forceinline__ void load_tile(const double *base, double (&o)[RY][CX], int ix0, int iy0,
                                          int nsx, int nsy)
{
    constexpr int sx = 16 * CX;
#pragma unroll
    for (int t = 0; t < RY; ++t) {
        const bool row = iy0 + t < nsy;
        const double *r = base + (size_t)(iy0 + t) * sx + ix0;
        if constexpr (CX % 2 == 0) {
#pragma unroll
            for (int q = 0; q < CX; q += 2) {
                double2 v = make_double2(0.0, 0.0);
                if (row) v = *reinterpret_cast<const double2 *>(r + q);
                o[t][q] = ix0 + q < nsx ? v.x : 0.0;
                o[t][q + 1] = ix0 + q + 1 < nsx ? v.y : 0.0;
            }
        } else {
#pragma unroll
            for (int q = 0; q < CX; ++q) o[t][q] = row && ix0 + q < nsx ? r[q] : 0.0;
        }
    }
}

__device__ __forceinline__ void stage_copy(const Ctx &c, const double *x, int n)
{
    typedef const __attribute__((address_space(1))) void *GPtr;
    typedef __attribute__((address_space(3))) void *LPtr;
    const int chunks = (n * 8 + 1023) / 1024;
    double *base = lds_ptr<double>(c, c.off.total);
    for (int ch = c.w; ch < chunks; ch += c.W) {
        int e = ch * 128 + c.lane * 2;
        e = e < n - 2 ? e : n - 2;
        __builtin_amdgcn_global_load_lds((GPtr)(x + e), (LPtr)(base + ch * 128), 16, 0, 0);
    }
}

__device__ __forceinline__ StageLoc jacobi_loc(int cur)
{
    StageLoc v{};
    v.src = v.xpb = v.xrb = v.lnb = v.lrb = cur;
    v.dst = cur ^ 1;
    v.omega = 1.0;
    v.box_at = -1;
    v.du_at = -1;
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

// The separable input factors gx [LX][nsx], gy [LY][nsy] into LDS (double and
// float copies), laid out for the tile: gx by padded column, gy by tile row.
template <int CX, int RY, int LX, int LY>
__device__ __forceinline__ void load_tables(Ctx &c, const double *gxs, const double *gys, int nsx,
                                            int nsy, bool sync = true)
{
    double *gx = lds_ptr<double>(c, c.off.gx);
    double *gy = lds_ptr<double>(c, c.off.gy);
    float *gxf = lds_ptr<float>(c, c.off.gxf);
    float *gyf = lds_ptr<float>(c, c.off.gyf);
    for (int t = c.tid; t < LX * 16 * CX; t += c.W * kWave) {
        const int aq = t >> 4, aa = aq / CX, ix = (t & 15) * CX + aq % CX;
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
    if (sync) __syncthreads();
}

// acc (thread 0 only): running bit-pattern max of (r_scaled, r_paper) over
// the stages processed with res_at == -1. WIDE: the residual's global reads
// of x_i, lambda_i, lambda_{i+1} and xref_i go through load_tile (16-byte
// loads; the batch kernel's 4-column tiles, where this saves memory
// instructions without spills; the other kernels and tiles keep element
// loads, which need fewer registers there).
template <typename T, int CX, int RY, int LX, int LY, bool WIDE = false>
__device__ __forceinline__ void stage_body(const IterArgs &a, const DevProblem &P,
                                           const StageLoc &v, Ctx &c,
                                           unsigned long long (&acc)[2])
{
    constexpr int M = LX * LY;
    const int n = P.n;
    double *uvec = lds_ptr<double>(c, c.off.uvec);
    double *kun = lds_ptr<double>(c, c.off.kun);
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
    double btl;   // (B^T lambda_i)_j in lane j < M
    {
        double xc[RY][CX], lc[RY][CX], Lx[RY][CX];
        if constexpr (WIDE) {   // the batch kernel: no prefetched slices
            load_tile<CX, RY>(Xc, xc, ix0, iy0, P.nsx, P.nsy);
            load_tile<CX, RY>(Lc, lc, ix0, iy0, P.nsx, P.nsy);
        } else {
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
        }
        if (c.tid < M) uvec[c.tid] = a.U[v.src][v.uo + (size_t)v.i * M + c.tid];
        if (v.tgx) load_tables<CX, RY, LX, LY>(c, v.tgx, v.tgy, P.nsx, P.nsy, false);
        if (v.xp_lds) stage_copy(c, Xp, n);   // x_{i-1}, requested with x_i
        __builtin_amdgcn_sched_barrier(0);
        nbsum<double, CX, RY>(xc, Lx, c);
        __builtin_amdgcn_sched_barrier(0);
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
            // the x_{i-1} copy has landed (this wave's part), and the
            // stencil's barrier publishes every wave's part
            if (v.xp_lds) __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_sched_barrier(0);
            nbsum<double, CX, RY>(g, Lg, c);
            __builtin_amdgcn_sched_barrier(0);
            double lnt[RY][CX], xrt[RY][CX];
            if constexpr (WIDE) {
                load_tile<CX, RY>(Xr, xrt, ix0, iy0, P.nsx, P.nsy);
                if (last) {
#pragma unroll
                    for (int t = 0; t < RY; ++t)
#pragma unroll
                        for (int q = 0; q < CX; ++q) lnt[t][q] = 0.0;
                } else {
                    load_tile<CX, RY>(Ln, lnt, ix0, iy0, P.nsx, P.nsy);
                }
            }
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) {
                    // nodes off the grid have no KKT row: their stencil of a
                    // valid neighbour is dropped (norms, right-hand sides)
                    double kl = 0.0, klr = 0.0;
                    if (valid(t, q)) {
                        const double ln = WIDE ? lnt[t][q] : (last ? 0.0 : Ln[pidx(t, q)]);
                        const double xr = WIDE ? xrt[t][q] : Xr[pidx(t, q)];
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
            __builtin_amdgcn_sched_barrier(0);
            b_apply<double, CX, RY, LX, LY>(uvec, c, Bu);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) {
                    double kx = 0.0, kxr = 0.0;
                    if (valid(t, q)) {
                        const double kk = P.k0 * (1.0 + P.k1 * xc[t][q]);
                        const double fx = h * (kk * Lx[t][q] + Bu[t][q]);
                        const double xp = v.xp_lds ? lds_ptr<double>(c, c.off.total)[pidx(t, q)]
                                                   : Xp[pidx(t, q)];
                        kx = xp - xc[t][q] + fx;
                        kxr = xdiff ? Xq[pidx(t, q)] - xc[t][q] + fx : kx;
                    }
                    mx = umax64(mx, abits(kxr));
                    b1[t][q] = T(kx);
                }
        }
        __builtin_amdgcn_sched_barrier(0);
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
        __builtin_amdgcn_sched_barrier(0);
        btl = bt_reduce<double, CX, RY, LX, LY>(lc, c, M);
        // every wave has read x_{i-1} from LDS (before bt_reduce's barrier):
        // the region now takes x_i for the update, copied during the lower layer
        if (v.xp_lds && !(a.residual_only || v.res_only)) stage_copy(c, Xc, n);
    }
    unsigned long long mu = 0;
    if (c.tid < M) {
        // with u~ = u^k the gamma term vanishes at evaluation; a stage whose
        // reference is another buffer's input (second sweep of SGS) keeps it
        double bg = 0.0;   // gradient of the input-box barrier
        if (P.tau > 0.0) bg = -P.tau / (uvec[c.tid] - P.ulo) + P.tau / (P.uhi - uvec[c.tid]);
        const double ku = h * (P.r * uvec[c.tid] + bg + btl);
        const double reg = v.utb >= 0
            ? P.gamma * (uvec[c.tid] - a.U[v.utb][v.uo + (size_t)v.i * M + c.tid]) : 0.0;
        kun[c.tid] = ku + reg;
        mu = abits(ku);
    }
    // the waves' norm partials go to LDS; thread 0 combines them after a
    // barrier: at once, or (defer_norms) after the lower layer's first one
    bool norms_owed = false;
    auto combine_norms = [&]() {
        if (norms_owed && c.tid == 0) {
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
        norms_owed = false;
    };
    if (want_res) {
        mx = wave_max64(mx, c.lane);
        ml = wave_max64(ml, c.lane);
        mu = wave_max64(mu, c.lane);
        if (c.lane == 0) {
            nrm[c.w * 4 + 0] = mx;
            nrm[c.w * 4 + 1] = ml;
            nrm[c.w * 4 + 2] = mu;
        }
        norms_owed = true;
        if (!v.defer_norms) {
            __syncthreads();
            combine_norms();
        }
    } else {
        __syncthreads();   // the norm path's barrier
    }
    // every wave has read its x_i, lambda_i (before the first stencil barrier):
    // the prefetch region may take the next stage's
    if (v.pnb >= 0) {
        const size_t sn = (size_t)v.so + (size_t)v.pni * n;
        prefetch_xl(c, a.X[v.pnb] + sn, a.LAM[v.pnb] + sn, n);
    }
    if (a.residual_only || v.res_only) {
        if (norms_owed) {
            __syncthreads();
            combine_norms();
        }
        return;
    }

    // ---- lower layer (T)
    const T hT = T(h), qT = T(P.q), c0T = T(P.c0);
    const double auu = h * P.r + P.gamma;
    T y5[RY][CX], y4[RY][CX];
    // v3 (the input step): element j in lane j < M of every wave (v3me) and as
    // wave-uniform values (v3s) for the applications of B
    double v3me = 0.0;
    T v3s[M];
#pragma unroll
    for (int j = 0; j < M; ++j) v3s[j] = T(0);
    for (int s = 0; s < a.n_schur; ++s) {
        T cc[RY][CX];
        if (s == 0) {
#pragma unroll
            for (int t = 0; t < RY; ++t)
#pragma unroll
                for (int q = 0; q < CX; ++q) cc[t][q] = -b1[t][q];
        } else {
            T Bv[RY][CX];
            b_apply<T, CX, RY, LX, LY>(v3s, c, Bv);
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
        const T bt = bt_reduce<T, CX, RY, LX, LY>(y4, c, M);
        if (s == 0) combine_norms();   // bt_reduce's barrier follows the partials
        // every wave forms v3 itself (same operands, same order): no barrier
        if (c.lane < M) {
            double au = auu;   // plus the barrier's Hessian with an input box
            if (P.tau > 0.0) {
                const double lo = uvec[c.lane] - P.ulo, hi = P.uhi - uvec[c.lane];
                au += h * (P.tau / (lo * lo) + P.tau / (hi * hi));
            }
            v3me = double((T(kun[c.lane]) + hT * bt) / T(au));
        }
        wave_bcast<T, M>(v3me, v3s);
    }
    if (norms_owed) {   // no Schur step ran
        __syncthreads();
        combine_norms();
    }
    {
        T cc[RY][CX];
        {
            T Bv[RY][CX];
            b_apply<T, CX, RY, LX, LY>(v3s, c, Bv);
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

    // ---- update S^{j+1} = S^j - omega ds (FP64); x_i, lam_i re-read (L2-resident)
    double *Xn = a.X[v.dst] + si;
    double *Lw = a.LAM[v.dst] + si;
    const double om = v.omega;
    const double *Xs = Xc;
    if (v.xp_lds) {   // x_i from the LDS copy
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        Xs = lds_ptr<double>(c, c.off.total);
    }
    if constexpr (WIDE) {
        // 16-byte stores of whole tile rows: the row padding receives zeros
#pragma unroll
        for (int t = 0; t < RY; ++t) {
            if (iy0 + t >= P.nsy) continue;
#pragma unroll
            for (int q = 0; q < CX; q += 2) {
                const int p = pidx(t, q);
                const bool v0 = ix0 + q < P.nsx, v1 = ix0 + q + 1 < P.nsx;
                const double x0v = v0 ? Xs[p] - om * double(y5[t][q]) : 0.0;
                const double x1v = v1 ? Xs[p + 1] - om * double(y5[t][q + 1]) : 0.0;
                const double l0v = v0 ? Lc[p] - om * double(y4[t][q]) : 0.0;
                const double l1v = v1 ? Lc[p + 1] - om * double(y4[t][q + 1]) : 0.0;
                *reinterpret_cast<double2 *>(Xn + p) = make_double2(x0v, x1v);
                *reinterpret_cast<double2 *>(Lw + p) = make_double2(l0v, l1v);
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < RY; ++t)
#pragma unroll
            for (int q = 0; q < CX; ++q)
                if (valid(t, q)) {
                    const int p = pidx(t, q);
                    Xn[p] = Xs[p] - om * double(y5[t][q]);
                    Lw[p] = Lc[p] - om * double(y4[t][q]);
                }
    }
    if (c.tid < M) {
        const double un = uvec[c.tid] - om * v3me;
        a.U[v.dst][v.uo + (size_t)v.i * M + c.tid] = un;
        if (v.du_at >= 0) {   // size of the FP64 correction step (reported per result)
            atomicMax(a.du + 2 * v.du_at, abits(om * v3me));
            atomicMax(a.du + 2 * v.du_at + 1, abits(un));
        }
    }
    if (P.tau > 0.0 && v.box_at >= 0) {
        // fraction-to-the-boundary limit of this stage's input step (eq.
        // eq_alphamax); the launch's box kernel takes the minimum over the
        // instance's stages and scales the steps when it is below 1
        double *lim = lds_ptr<double>(c, c.off.red);
        if (c.tid < M) {
            const double u = uvec[c.tid], d = v3me;
            double l = 1.0;
            if (d > 0.0) l = 0.995 * (u - P.ulo) / d;
            else if (d < 0.0) l = 0.995 * (P.uhi - u) / (-d);
            lim[c.tid] = fmax(l, 0.0);   // S^j is strictly feasible: l > 0
        }
        __syncthreads();
        if (c.tid == 0) {
            double l = 1.0;
            for (int j = 0; j < M; ++j) l = fmin(l, lim[j]);
            a.apart[v.box_at] = l;
        }
    }
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
