// nmpc_net.hip -- kernels of the learned warm start: a patch encoder mapping
// second-order features of (x0, xref) windows around each actuator to that
// actuator's input trajectory.
//
// The hidden layers are GEMMs on bf16 operands with fp32 accumulation on the
// matrix cores (v_mfma_f32_16x16x32_bf16), so forward, data gradient and
// weight gradient are the three operand layouts of one kernel:
//   forward  C = X W          (A [M][K], B [K][N])
//   dgrad    C = dY W^T       (B stored [N][K])
//   wgrad    C = X^T dY       (A stored [K][M])
// The per-actuator linear map of the second-order features runs on fp32
// operands (v_mfma_f32_16x16x4_f32). The small elementwise kernels (feature
// gather, ReLU gradient, column sums,
// squared-error gradient, Adam, layout packing) complete the training step.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmpc_net.h"

namespace nmpc {

using bf16x8 = __attribute__((ext_vector_type(8))) __bf16;
using f32x4 = __attribute__((ext_vector_type(4))) float;

__device__ __forceinline__ unsigned short f2bf(float f)
{
    // round to nearest even; NaN stays NaN
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned int)b << 16); }

// ------------------------------------------------------------------- GEMM

constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;

// C[m][n] = beta C + sum_k A(m, k) B(k, n) (+ bias[n]) (ReLU); outputs fp32 C
// and/or bf16 Cb. A(m, k) = TA ? A[k lda + m] : A[m lda + k];
// B(k, n) = TB ? B[n ldb + k] : B[k ldb + n]. Tails are zero-filled.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm(const GemmArgs g)
{
    __shared__ __align__(16) unsigned short As[kBM][kBK + kPad];   // [m][k]
    __shared__ __align__(16) unsigned short Bs[kBN][kBK + kPad];   // [n][k]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    // split K: this workgroup's part [kb, ke) (kc a multiple of kBK)
    const int kb = g.ksplit > 1 ? blockIdx.z * g.kc : 0;
    const int ke = g.ksplit > 1 ? min(g.K, kb + g.kc) : g.K;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // each thread stages 8 consecutive elements of A and of B per K step; when
    // they are contiguous in memory, inside the matrix and 16-byte aligned,
    // as one 16-byte load
    const bool vecA = !TA && (g.lda & 7) == 0 && (((uintptr_t)g.A) & 15) == 0;
    const bool vecB = !TB && (g.ldb & 7) == 0 && (((uintptr_t)g.B) & 15) == 0;
    for (int k0 = kb; k0 < ke; k0 += kBK) {
        // stage a 64 x 32 tile of A and of B^T (8 elements per thread each)
        {
            const int r0 = (tid * 8) / kBK, kk0 = (tid * 8) % kBK;   // !TA: 8 consecutive k
            if (vecA && m0 + r0 < g.M && k0 + kk0 + 8 <= ke) {
                const uint4 q = *(const uint4 *)&g.A[(size_t)(m0 + r0) * g.lda + k0 + kk0];
                *(uint4 *)&As[r0][kk0] = q;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int idx = tid * 8 + e;
                    int r, kk;
                    if (TA) { kk = idx / kBM; r = idx % kBM; }   // consecutive threads walk m
                    else    { r = idx / kBK; kk = idx % kBK; }   // consecutive threads walk k
                    const int gm = m0 + r, gk = k0 + kk;
                    unsigned short v = 0;
                    if (gm < g.M && gk < ke) v = TA ? g.A[(size_t)gk * g.lda + gm] : g.A[(size_t)gm * g.lda + gk];
                    As[r][kk] = v;
                }
            }
        }
        {
            const int kk0 = (tid * 8) / kBN, c0 = (tid * 8) % kBN;   // !TB: 8 consecutive n
            if (vecB && k0 + kk0 < ke && n0 + c0 + 8 <= g.N) {
                const uint4 q = *(const uint4 *)&g.B[(size_t)(k0 + kk0) * g.ldb + n0 + c0];
                const unsigned short *qs = (const unsigned short *)&q;
#pragma unroll
                for (int e = 0; e < 8; ++e) Bs[c0 + e][kk0] = qs[e];
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int idx = tid * 8 + e;
                    int c, kk;
                    if (TB) { c = idx / kBK; kk = idx % kBK; }   // consecutive threads walk k
                    else    { kk = idx / kBN; c = idx % kBN; }   // consecutive threads walk n
                    const int gn = n0 + c, gk = k0 + kk;
                    unsigned short v = 0;
                    if (gn < g.N && gk < ke) v = TB ? g.B[(size_t)gn * g.ldb + gk] : g.B[(size_t)gk * g.ldb + gn];
                    Bs[c][kk] = v;
                }
            }
        }
        __syncthreads();
        {
            // gfx950's 16 x 16 x 32 bf16 MFMA, one per block and K step:
            // lane l holds row / column l % 16 and k = 8 (l / 16) .. + 7
            const int kq = 8 * (lane >> 4);
            bf16x8 af[2], bfr[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                __builtin_memcpy(&af[i], &As[wm + i * 16 + (lane & 15)][kq], 16);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                __builtin_memcpy(&bfr[j], &Bs[wn + j * 16 + (lane & 15)][kq], 16);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // result: lane l holds rows 4 (l / 16) + r, column l % 16 of each 16 x 16 block
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
                const int gn = n0 + wn + j * 16 + (lane & 15);
                if (gm >= g.M || gn >= g.N) continue;
                float v = acc[i][j][r];
                if (g.ksplit > 1) {   // raw partial; k_gemm_reduce applies the epilogue
                    g.work[((size_t)blockIdx.z * g.M + gm) * g.N + gn] = v;
                    continue;
                }
                if (g.C && g.beta != 0.f) v += g.beta * g.C[(size_t)gm * g.ldc + gn];
                if (g.bias) v += g.bias[gn];
                if (g.relu) v = v > 0.f ? v : 0.f;
                if (g.C) g.C[(size_t)gm * g.ldc + gn] = v;
                if (g.Cb) g.Cb[(size_t)gm * g.ldcb + gn] = f2bf(v);
            }
}

// Split-K epilogue of k_gemm: the parts summed in a fixed order, then beta C,
// the bias, the ReLU and the fp32 / bf16 outputs. One thread per (m, n).
__global__ void k_gemm_reduce(const GemmArgs g)
{
    const size_t mn = (size_t)g.M * g.N;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= mn) return;
    const int gm = (int)(t / g.N), gn = (int)(t % g.N);
    float v = 0.f;
    for (int p = 0; p < g.ksplit; ++p) v += g.work[(size_t)p * mn + t];
    if (g.C && g.beta != 0.f) v += g.beta * g.C[(size_t)gm * g.ldc + gn];
    if (g.bias) v += g.bias[gn];
    if (g.relu) v = v > 0.f ? v : 0.f;
    if (g.C) g.C[(size_t)gm * g.ldc + gn] = v;
    if (g.Cb) g.Cb[(size_t)gm * g.ldcb + gn] = f2bf(v);
}

// Grouped GEMM on the matrix cores with fp32 or fp64 products: the
// per-actuator linear map of the network's second-order features (fp32
// operands, v_mfma_f32_16x16x4_f32: more significant bits than bf16 carries)
// and the fit of that map by its normal equations (fp64 products and
// accumulation, v_mfma_f64_16x16x4_f64, on fp32 or fp64 operands). Group z
// works on A + z sa, B + z sb, Cin + z sc, C + z sc.
// A(m, k) = TA ? A[k lda + m] : A[m lda + k]; B(k, n) = B[k ldb + n];
// C = alpha A B + beta Cin (Cin = C when not given). Tails are zero-filled.
constexpr int kFK = 16;

template <typename T> struct MfmaTile;
// Result layout of one 16 x 16 block: lane l holds column l % 16 and rows
// row(l, r), r = 0..3 (fp32: 4 consecutive rows per lane quarter; fp64: rows
// interleaved with stride 4).
template <> struct MfmaTile<float> {
    using acc_t = f32x4;
    static constexpr int pad = 4;
    __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
    __device__ static acc_t mma(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct MfmaTile<double> {
    using acc_t = __attribute__((ext_vector_type(4))) double;
    static constexpr int pad = 1;
    __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
    __device__ static acc_t mma(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

template <bool TA, typename InT, typename AccT>
__global__ void __launch_bounds__(256) k_gemm_mx(const GemmMxArgs g)
{
    using MT = MfmaTile<AccT>;
    __shared__ AccT As[kBM][kFK + MT::pad];   // [m][k]
    __shared__ AccT Bs[kBN][kFK + MT::pad];   // [n][k]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    // blockIdx.z = group * ksplit + part: part covers K range [kb, ke)
    const int grp = blockIdx.z / g.ksplit, part = blockIdx.z % g.ksplit;
    const int kb = part * g.kc, ke = min(g.K, kb + g.kc);
    const InT *A = (const InT *)g.A + (size_t)grp * g.sa;
    const InT *B = (const InT *)g.B + (size_t)grp * g.sb;
    AccT *C = (AccT *)g.C + (size_t)grp * g.sc;
    const AccT *Cin = (g.Cin ? (const AccT *)g.Cin : (const AccT *)g.C) + (size_t)grp * g.sc;
    typename MT::acc_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = typename MT::acc_t{0, 0, 0, 0};

    for (int k0 = kb; k0 < ke; k0 += kFK) {
        // a 64 x 16 tile of A and of B^T: four elements per thread each
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid * 4 + e;
            int r, kk;
            if (TA) { kk = idx / kBM; r = idx % kBM; }   // consecutive threads walk m
            else    { r = idx / kFK; kk = idx % kFK; }   // consecutive threads walk k
            const int gm = m0 + r, gk = k0 + kk;
            AccT v = 0;
            if (gm < g.M && gk < ke) v = (AccT)(TA ? A[(size_t)gk * g.lda + gm] : A[(size_t)gm * g.lda + gk]);
            As[r][kk] = v;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid * 4 + e;
            const int kk = idx / kBN, c = idx % kBN;         // consecutive threads walk n
            const int gn = n0 + c, gk = k0 + kk;
            Bs[c][kk] = (gn < g.N && gk < ke) ? (AccT)B[(size_t)gk * g.ldb + gn] : (AccT)0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kFK; ks += 4) {
            // lane l holds row / column l % 16 at k = ks + l / 16
            const int kq = ks + (lane >> 4);
            AccT af[2], bfr[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = As[wm + i * 16 + (lane & 15)][kq];
#pragma unroll
            for (int j = 0; j < 2; ++j) bfr[j] = Bs[wn + j * 16 + (lane & 15)][kq];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = MT::mma(af[i], bfr[j], acc[i][j]);
        }
        __syncthreads();
    }
    const AccT alpha = (AccT)g.alpha, beta = (AccT)g.beta;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + i * 16 + MT::row(lane, r);
                const int gn = n0 + wn + j * 16 + (lane & 15);
                if (gm >= g.M || gn >= g.N) continue;
                if (g.ksplit > 1) {   // partial sum of this K range: [group][part][M][N]
                    ((AccT *)g.work)[((size_t)blockIdx.z * g.M + gm) * g.N + gn] = acc[i][j][r];
                    continue;
                }
                AccT v = alpha * acc[i][j][r];
                if (beta != (AccT)0) v += beta * Cin[(size_t)gm * g.ldc + gn];
                C[(size_t)gm * g.ldc + gn] = v;
            }
}

// Split-K epilogue: C_g = alpha sum_part work[g][part] + beta Cin_g, the parts
// added in a fixed order. One thread per (group, m, n).
template <typename AccT>
__global__ void k_splitk_reduce(const GemmMxArgs g)
{
    const size_t mn = (size_t)g.M * g.N, tot = mn * (size_t)gridDim.y;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= mn) return;
    const int grp = blockIdx.y;
    const int m = (int)(t / g.N), n = (int)(t % g.N);
    const AccT *wk = (const AccT *)g.work + (size_t)grp * g.ksplit * mn + t;
    AccT v = 0;
    for (int p = 0; p < g.ksplit; ++p) v += wk[(size_t)p * mn];
    AccT *C = (AccT *)g.C + (size_t)grp * g.sc;
    const AccT *Cin = (g.Cin ? (const AccT *)g.Cin : (const AccT *)g.C) + (size_t)grp * g.sc;
    v *= (AccT)g.alpha;
    if (g.beta != 0.0) v += (AccT)g.beta * Cin[(size_t)m * g.ldc + n];
    C[(size_t)m * g.ldc + n] = v;
    (void)tot;
}

// Normal equations of group z: G_z (n x n, row stride ld) gets the ridge
// rel * trace(G_z) / n added to its diagonal, and X_z = I / trace(G_z + ridge)
// starts the Newton-Schulz inverse iteration X <- 2 X - X G X (the trace bounds
// the largest eigenvalue of a positive semidefinite matrix, so the iteration
// contracts). One workgroup per group; X rows have stride ld.
__global__ void __launch_bounds__(1024) k_ls_prepare(double *G, int n, int ld, long long sg,
                                                     double rel, double *X, long long sx)
{
    __shared__ double part[1024];
    double *Gz = G + (size_t)blockIdx.x * sg;
    double *Xz = X + (size_t)blockIdx.x * sx;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += Gz[(size_t)i * ld + i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    const double tr = part[0];
    const double ridge = rel * tr / n;
    const double a = 1.0 / (tr + n * ridge);
    for (int i = threadIdx.x; i < n; i += blockDim.x) Gz[(size_t)i * ld + i] += ridge;
    for (size_t t = threadIdx.x; t < (size_t)n * n; t += blockDim.x) {
        const int i = (int)(t / n), j = (int)(t % n);
        Xz[(size_t)i * ld + j] = i == j ? a : 0.0;
    }
}

// ------------------------------------------------------------ elementwise

// Input rows of the network. For instance b and actuator p = pb * L + pa of
// an L x L lattice on an ns x ns grid, a win x win window starting
// (win - s) / 2 nodes before the actuator's cell (s = ns / L), in `planes`
// feature planes of the scaled fields xt = x0 / 0.1 - 1 and rt = xref / 0.3:
// xt, rt, xt^2 - 1/3, xt rt, rt^2 - 1/3 (the first two, or all five); zero
// outside the grid. Then a one-hot actuator index and zeros up to the row
// length ld. Row b * L^2 + p; fp32 (Xf) and/or bf16 (Xb) copies.
// One workgroup per row: each thread takes window pixels, reads x0 and xref
// once per pixel and writes the pixel's value in every plane (consecutive
// pixels of a plane are consecutive columns, so the stores coalesce).
__global__ void k_features(const FeatArgs a)
{
    const int row = blockIdx.x;
    const int LL = a.L * a.L, b = row / LL, p = row % LL;
    const int ww = a.win * a.win, feat = a.planes * ww;
    const int s = a.ns / a.L, off = (a.win - s) / 2;
    const int iy0 = (p / a.L) * s - off, ix0 = (p % a.L) * s - off;
    const size_t base = (size_t)row * a.ld;
    const double *x0 = a.x0 + (size_t)b * a.ns * a.ns, *xr = a.xref + (size_t)b * a.ns * a.ns;
    auto put = [&](int col, float v) {
        if (a.Xf) a.Xf[base + col] = v;
        if (a.Xb) a.Xb[base + col] = f2bf(v);
    };
    for (int r = threadIdx.x; r < ww; r += blockDim.x) {
        const int iy = iy0 + r / a.win, ix = ix0 + r % a.win;
        double xt = 0.0, rt = 0.0;
        const bool in = iy >= 0 && iy < a.ns && ix >= 0 && ix < a.ns;
        if (in) {
            const int gi = iy * a.ns + ix;
            xt = x0[gi] / 0.1 - 1.0;
            rt = xr[gi] / 0.3;
        }
        put(r, in ? (float)xt : 0.f);
        put(ww + r, in ? (float)rt : 0.f);
        if (a.planes == 5) {
            put(2 * ww + r, in ? (float)(__dmul_rn(xt, xt) - 1.0 / 3.0) : 0.f);
            put(3 * ww + r, in ? (float)__dmul_rn(xt, rt) : 0.f);
            put(4 * ww + r, in ? (float)(__dmul_rn(rt, rt) - 1.0 / 3.0) : 0.f);
        }
    }
    for (int col = feat + threadIdx.x; col < a.ld; col += blockDim.x)
        put(col, col - feat == p ? 1.f : 0.f);
}

// Forward pass of the per-actuator map with the features gathered in place
// (no feature rows in HBM). Workgroup (instance tile of 64, K part, actuator
// p): for each 32-pixel chunk of the window a thread loads x0 and xref of one
// pixel for 8 instances (a wave's lanes read consecutive pixels) and a
// contiguous slice of the chunk's Ws rows for every plane; then per plane the
// feature values (the same arithmetic as k_features) and the Ws rows go
// through LDS into v_mfma_f32_16x16x4_f32 (each wave 16 instances x 48
// columns, N <= 48). The one-hot column's contribution, the row
// Ws[p][planes win^2 + p], is added by part 0. Partial sums [p][part][b][n]
// are summed in a fixed order by k_splitk_reduce.
constexpr int kMapBM = 64, kMapBN = 48, kMapKC = 32;

__global__ void __launch_bounds__(256) k_map_fwd(const MapArgs a)
{
    __shared__ float As[kMapBM][kMapKC + 4];   // [instance][pixel]
    __shared__ float Bs[kMapBN][kMapKC + 4];   // [column][pixel]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.x * kMapBM, part = blockIdx.y, p = blockIdx.z;
    const int ww = a.win * a.win, feat = a.planes * ww;
    const int s = a.ns / a.L, off = (a.win - s) / 2;
    const int iy0 = (p / a.L) * s - off, ix0 = (p % a.L) * s - off;
    const float *W = a.Ws + (size_t)p * a.K0 * a.N;
    const int kk = tid & (kMapKC - 1), q0 = tid >> 5;   // A: pixel kk of instances q0 + 8 q
    const size_t img = (size_t)a.ns * a.ns;
    f32x4 acc[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int c0 = part * a.cpp, c1 = min(a.chunks, c0 + a.cpp);
    for (int c = c0; c < c1; ++c) {
        const int r = c * kMapKC + kk;
        const int iy = iy0 + r / a.win, ix = ix0 + r % a.win;
        const bool pix = r < ww && iy >= 0 && iy < a.ns && ix >= 0 && ix < a.ns;
        const int gi = pix ? iy * a.ns + ix : 0;
        double xt[8], rt[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int gm = m0 + q0 + 8 * q;
            xt[q] = 0.0; rt[q] = 0.0;
            if (pix && gm < a.count) {
                xt[q] = a.x0[(size_t)gm * img + gi] / 0.1 - 1.0;
                rt[q] = a.xref[(size_t)gm * img + gi] / 0.3;
            }
        }
        // the chunk's Ws rows of a plane are one contiguous block of kr * N floats
        const int kr = min(kMapKC, ww - c * kMapKC), nb = kr * a.N;
        float bv[5][6];
#pragma unroll
        for (int ch = 0; ch < 5; ++ch)
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const int idx = tid + 256 * e;
                bv[ch][e] = (ch < a.planes && idx < nb)
                                ? W[(size_t)(ch * ww + c * kMapKC) * a.N + idx] : 0.f;
            }
#pragma unroll
        for (int ch = 0; ch < 5; ++ch) {
            if (ch >= a.planes) break;
            __syncthreads();   // the previous plane's fragments are read
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                double f;
                switch (ch) {
                case 0: f = xt[q]; break;
                case 1: f = rt[q]; break;
                case 2: f = __dmul_rn(xt[q], xt[q]) - 1.0 / 3.0; break;
                case 3: f = __dmul_rn(xt[q], rt[q]); break;
                default: f = __dmul_rn(rt[q], rt[q]) - 1.0 / 3.0; break;
                }
                const bool in = pix && m0 + q0 + 8 * q < a.count;
                As[q0 + 8 * q][kk] = in ? (float)f : 0.f;
            }
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const int idx = tid + 256 * e;
                if (idx < kMapKC * kMapBN) {
                    const int k = idx / a.N, n = idx % a.N;
                    if (k < kMapKC) Bs[n][k] = idx < nb ? bv[ch][e] : 0.f;
                }
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < kMapKC; ks += 4) {
                const int kq = ks + (lane >> 4);
                const float af = As[w * 16 + (lane & 15)][kq];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int n = j * 16 + (lane & 15);
                    const float bf = n < a.N ? Bs[n][kq] : 0.f;
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bf, acc[j], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = m0 + w * 16 + 4 * (lane >> 4) + r, n = j * 16 + (lane & 15);
            if (m >= a.count || n >= a.N) continue;
            float v = acc[j][r];
            if (part == 0) v += W[(size_t)(feat + p) * a.N + n];
            a.work[(((size_t)p * a.ksplit + part) * a.count + m) * a.N + n] = v;
        }
}

// dH = dH * (H > 0), also as bf16.
__global__ void k_relu_grad(float *dh, const float *hact, unsigned short *dhb, long long n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)n; t += stride) {
        const float v = hact[t] > 0.f ? dh[t] : 0.f;
        dh[t] = v;
        dhb[t] = f2bf(v);
    }
}

// out[n] = sum_m A[m][n] (one thread per column, fixed summation order).
__global__ void k_colsum(const float *A, int M, int N, int lda, float *out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += A[(size_t)m * lda + n];
    out[n] = s;
}

// dY = scale (Y - T) (fp32 and bf16) and per-row squared-error partials.
__global__ void k_mse(const float *Y, int ldy, const float *T, int ldt, int M, int N, float scale,
                      float *dY, unsigned short *dYb, int lddy, float *row_sse)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    float s = 0.f;
    for (int n = 0; n < N; ++n) {
        const float e = Y[(size_t)m * ldy + n] - T[(size_t)m * ldt + n];
        s += e * e;
        const float g = scale * e;
        dY[(size_t)m * lddy + n] = g;
        dYb[(size_t)m * lddy + n] = f2bf(g);
    }
    row_sse[m] = s;
}

// Adam on fp32 master weights (decoupled weight decay), refreshing the bf16 copy.
__global__ void k_adam(const AdamArgs a)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const float c1 = 1.f - powf(a.b1, (float)a.step), c2 = 1.f - powf(a.b2, (float)a.step);
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)a.n; t += stride) {
        const float g = a.g[t];
        const float m = a.b1 * a.m[t] + (1.f - a.b1) * g;
        const float v = a.b2 * a.v[t] + (1.f - a.b2) * g * g;
        a.m[t] = m;
        a.v[t] = v;
        float w = a.w[t] * (1.f - a.lr * a.wd);
        w -= a.lr * (m / c1) / (sqrtf(v / c2) + a.eps);
        a.w[t] = w;
        if (a.wb) a.wb[t] = f2bf(w);
    }
}

__global__ void k_to_bf16(const float *x, unsigned short *y, long long n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)n; t += stride)
        y[t] = f2bf(x[t]);
}

// u [count][N][m] (double) <-> rows [count * m][ldr] of N values (float), scaled.
__global__ void k_pack_u(const double *u, int count, int N, int m, float scale, float *rows, int ldr)
{
    const size_t tot = (size_t)count * N * m, stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
        const size_t b = t / ((size_t)N * m), r = t % ((size_t)N * m);
        const int i = (int)(r / m), j = (int)(r % m);
        rows[(b * m + j) * ldr + i] = float(u[t]) * scale;
    }
}
__global__ void k_unpack_u(const float *rows, int ldr, int count, int N, int m, float scale, double *u)
{
    const size_t tot = (size_t)count * N * m, stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
        const size_t b = t / ((size_t)N * m), r = t % ((size_t)N * m);
        const int i = (int)(r / m), j = (int)(r % m);
        u[t] = double(rows[(b * m + j) * ldr + i]) * scale;
    }
}

const void *gemm_kernel(int ta, int tb)
{
    if (!ta && !tb) return (const void *)&k_gemm<false, false>;
    if (!ta && tb) return (const void *)&k_gemm<false, true>;
    if (ta && !tb) return (const void *)&k_gemm<true, false>;
    return (const void *)&k_gemm<true, true>;
}
const void *features_kernel() { return (const void *)&k_features; }
const void *map_fwd_kernel() { return (const void *)&k_map_fwd; }
const void *gemm_mx_kernel(int ta, int in64, int acc64)
{
    if (!acc64) return ta ? (const void *)&k_gemm_mx<true, float, float>
                          : (const void *)&k_gemm_mx<false, float, float>;
    if (in64) return ta ? (const void *)&k_gemm_mx<true, double, double>
                        : (const void *)&k_gemm_mx<false, double, double>;
    return ta ? (const void *)&k_gemm_mx<true, float, double>
              : (const void *)&k_gemm_mx<false, float, double>;
}
const void *ls_prepare_kernel() { return (const void *)&k_ls_prepare; }
const void *splitk_reduce_kernel() { return (const void *)&k_splitk_reduce<float>; }
const void *gemm_reduce_kernel() { return (const void *)&k_gemm_reduce; }
const void *relu_grad_kernel() { return (const void *)&k_relu_grad; }
const void *colsum_kernel() { return (const void *)&k_colsum; }
const void *mse_kernel() { return (const void *)&k_mse; }
const void *adam_kernel() { return (const void *)&k_adam; }
const void *to_bf16_kernel() { return (const void *)&k_to_bf16; }
const void *pack_u_kernel() { return (const void *)&k_pack_u; }
const void *unpack_u_kernel() { return (const void *)&k_unpack_u; }

}  // namespace nmpc
