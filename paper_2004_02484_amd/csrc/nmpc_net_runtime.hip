// nmpc_net_runtime.hip -- C ABI of the warm-start network kernels: argument
// checks and launches on the caller's stream (all pointers are device memory).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "nmpc.h"
#include "nmpc_net.h"

namespace {

int net_fail(int code, const char *msg)
{
    nmpc_set_last_error(msg);
    return code;
}

#define NET_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return net_fail(NMPC_E_DEVICE, hipGetErrorString(e_));    \
    } while (0)

unsigned grid_for(size_t tot) { return (unsigned)std::min<size_t>((tot + 255) / 256 + 1, 16384); }

int launch_mx(int ta, int in64, int acc64, int32_t M, int32_t N, int32_t K, const void *A,
              int32_t lda, int64_t sa, const void *B, int32_t ldb, int64_t sb, double alpha,
              double beta, const void *Cin, void *C, int32_t ldc, int64_t sc, int32_t groups,
              void *stream, const char *what, int32_t ksplit = 1, void *work = nullptr)
{
    if (M < 1 || N < 1 || K < 1 || groups < 1 || !A || !B || !C || ksplit < 1 ||
        (long long)groups * ksplit > 65535 || (ksplit > 1 && !work))
        return net_fail(NMPC_E_ARG, what);
    if (lda < (ta ? M : K) || ldb < N || ldc < N) return net_fail(NMPC_E_ARG, what);
    if (groups > 1 && (sa < 0 || sb < 0 || sc < 0)) return net_fail(NMPC_E_ARG, what);
    // K parts: multiples of the 16-deep K step
    const int kc = ksplit > 1 ? ((K + ksplit - 1) / ksplit + 15) / 16 * 16 : K;
    nmpc::GemmMxArgs g{M, N, K, A, lda, B, ldb, alpha, beta, Cin, C, ldc, (long long)sa,
                       (long long)sb, (long long)sc, ksplit, kc, work};
    void *args[] = {(void *)&g};
    NET_TRY(hipLaunchKernel(nmpc::gemm_mx_kernel(ta != 0, in64, acc64),
                            dim3((N + 63) / 64, (M + 63) / 64, groups * ksplit), dim3(256), args,
                            0, (hipStream_t)stream));
    if (ksplit > 1) {
        const size_t mn = (size_t)M * N;
        NET_TRY(hipLaunchKernel(nmpc::splitk_reduce_kernel(), dim3((unsigned)((mn + 255) / 256), groups),
                                dim3(256), args, 0, (hipStream_t)stream));
    }
    return NMPC_OK;
}

// Split-K partials of nmpc_gemm_f32_noalloc: a file-scope device array, one
// copy per GPU, held until the process ends. Host code must not pass the
// array's name to a kernel (on the host it is only a stand-in): the device
// address of each GPU's copy is looked up once per device and kept here.
constexpr size_t kNoAllocFloats = (size_t)2 << 20;   // 8 MiB
static __device__ __align__(256) float scratch[kNoAllocFloats];
constexpr int kMaxDevices = 64;
float *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

int scratch_for_current_device(float **out)
{
    int dev = -1;
    NET_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return net_fail(NMPC_E_DEVICE, "gemm_f32_noalloc: device index");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return net_fail(NMPC_E_DEVICE, "gemm_f32_noalloc: hipGetSymbolAddress of the scratch array failed");
        g_scratch_ptr[dev] = (float *)p;
    }
    *out = g_scratch_ptr[dev];
    return NMPC_OK;
}

}  // namespace

namespace nmpc {

int gemm_bf16_split(int ta, int tb, int M, int N, int K, const uint16_t *A, int lda, const uint16_t *B,
                    int ldb, float beta, float *C, int ldc, const float *bias, int relu, uint16_t *Cb,
                    int ldcb, int ksplit, float *work, void *stream)
{
    if (M < 1 || N < 1 || K < 1 || !A || !B || (!C && !Cb))
        return net_fail(NMPC_E_ARG, "gemm: bad sizes or NULL operand");
    if (lda < (ta ? M : K) || ldb < (tb ? K : N) || (C && ldc < N) || (Cb && ldcb < N))
        return net_fail(NMPC_E_ARG, "gemm: leading dimension too small");
    if (beta != 0.f && !C) return net_fail(NMPC_E_ARG, "gemm: beta needs C");
    if (ksplit < 1 || (ksplit > 1 && !work)) return net_fail(NMPC_E_ARG, "gemm: split K needs a workspace");
    // parts of a whole number of 32-wide K steps; no empty part
    const int steps = (K + 31) / 32;
    ksplit = std::min(ksplit, steps);
    const int kc = (steps + ksplit - 1) / ksplit * 32;
    ksplit = (K + kc - 1) / kc;
    GemmArgs g{M, N, K, A, lda, B, ldb, beta, C, ldc, bias, relu ? 1 : 0, Cb, ldcb, ksplit, kc, work};
    void *args[] = {(void *)&g};
    NET_TRY(hipLaunchKernel(gemm_kernel(ta != 0, tb != 0), dim3((N + 63) / 64, (M + 63) / 64, ksplit),
                            dim3(256), args, 0, (hipStream_t)stream));
    if (ksplit > 1)
        NET_TRY(hipLaunchKernel(gemm_reduce_kernel(), dim3((unsigned)(((size_t)M * N + 255) / 256)),
                                dim3(256), args, 0, (hipStream_t)stream));
    return NMPC_OK;
}

int map_forward(const double *x0, const double *xref, int count, int ns, int L, int win, int planes,
                const float *Ws, int K0, int N, float beta, float *Y, float *work, void *stream)
{
    if (!x0 || !xref || !Ws || !Y || !work || count < 1 || ns < 1 || L < 1 || L > 8 || ns % L ||
        win < ns / L || (win - ns / L) % 2 || (planes != 2 && planes != 5) || N < 1 || N > 48 ||
        K0 < planes * win * win + L * L)
        return net_fail(NMPC_E_ARG, "map_forward: bad arguments");
    const int chunks = (win * win + 31) / 32;
    int ksplit = std::min(8, chunks);
    const int cpp = (chunks + ksplit - 1) / ksplit;
    ksplit = (chunks + cpp - 1) / cpp;   // no empty part
    MapArgs a{x0, xref, count, ns, L, win, planes, Ws, K0, N, chunks, cpp, ksplit, work};
    void *args[] = {(void *)&a};
    NET_TRY(hipLaunchKernel(map_fwd_kernel(), dim3((count + 63) / 64, ksplit, L * L), dim3(256), args,
                            0, (hipStream_t)stream));
    // the parts summed in a fixed order, beta Y added (row stride L^2 N, group stride N)
    GemmMxArgs g{count, N, K0, nullptr, 0, nullptr, 0, 1.0, (double)beta, nullptr, Y, L * L * N,
                 0, 0, (long long)N, ksplit, 0, work};
    void *rargs[] = {(void *)&g};
    NET_TRY(hipLaunchKernel(splitk_reduce_kernel(), dim3((unsigned)(((size_t)count * N + 255) / 256), L * L),
                            dim3(256), rargs, 0, (hipStream_t)stream));
    return NMPC_OK;
}

}  // namespace nmpc

extern "C" {

int nmpc_gemm_bf16(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K,
                   const uint16_t *A, int32_t lda, const uint16_t *B, int32_t ldb, float beta,
                   float *C, int32_t ldc, const float *bias, int32_t relu, uint16_t *Cb,
                   int32_t ldcb, void *stream)
{
    return nmpc::gemm_bf16_split(trans_a, trans_b, M, N, K, A, lda, B, ldb, beta, C, ldc, bias, relu,
                                 Cb, ldcb, 1, nullptr, stream);
}

int nmpc_gemm_f32(int32_t trans_a, int32_t M, int32_t N, int32_t K, const float *A, int32_t lda,
                  int64_t stride_a, const float *B, int32_t ldb, int64_t stride_b, float beta,
                  float *C, int32_t ldc, int64_t stride_c, int32_t groups, int32_t ksplit,
                  float *work, void *stream)
{
    return launch_mx(trans_a, 0, 0, M, N, K, A, lda, stride_a, B, ldb, stride_b, 1.0, beta,
                     nullptr, C, ldc, stride_c, groups, stream, "gemm_f32: bad arguments", ksplit,
                     work);
}

int nmpc_gemm_f32_noalloc(int32_t trans_a, int32_t M, int32_t N, int32_t K, const float *A,
                          int32_t lda, int64_t stride_a, const float *B, int32_t ldb,
                          int64_t stride_b, float beta, float *C, int32_t ldc, int64_t stride_c,
                          int32_t groups, int32_t ksplit, void *stream)
{
    if (M < 1 || N < 1 || groups < 1 || ksplit < 1)
        return net_fail(NMPC_E_ARG, "gemm_f32_noalloc: bad arguments");
    float *work = nullptr;
    if (ksplit > 1) {
        const unsigned long long need =
            (unsigned long long)groups * (unsigned long long)ksplit * (unsigned long long)M * N;
        if (need > kNoAllocFloats)
            return net_fail(NMPC_E_ARG, "gemm_f32_noalloc: groups * ksplit * M * N exceeds the "
                                        "static scratch of 2^21 floats (8 MiB)");
        const int rc = scratch_for_current_device(&work);
        if (rc) return rc;
    }
    return launch_mx(trans_a, 0, 0, M, N, K, A, lda, stride_a, B, ldb, stride_b, 1.0, beta,
                     nullptr, C, ldc, stride_c, groups, stream, "gemm_f32_noalloc: bad arguments",
                     ksplit, work);
}

int nmpc_gemm_f64(int32_t trans_a, int32_t M, int32_t N, int32_t K, const double *A, int32_t lda,
                  int64_t stride_a, const double *B, int32_t ldb, int64_t stride_b, double alpha,
                  double beta, const double *Cin, double *C, int32_t ldc, int64_t stride_c,
                  int32_t groups, void *stream)
{
    return launch_mx(trans_a, 1, 1, M, N, K, A, lda, stride_a, B, ldb, stride_b, alpha, beta,
                     Cin, C, ldc, stride_c, groups, stream, "gemm_f64: bad arguments");
}

int nmpc_gemm_f32_acc64(int32_t trans_a, int32_t M, int32_t N, int32_t K, const float *A,
                        int32_t lda, int64_t stride_a, const float *B, int32_t ldb,
                        int64_t stride_b, double beta, double *C, int32_t ldc, int64_t stride_c,
                        int32_t groups, void *stream)
{
    return launch_mx(trans_a, 0, 1, M, N, K, A, lda, stride_a, B, ldb, stride_b, 1.0, beta,
                     nullptr, C, ldc, stride_c, groups, stream, "gemm_f32_acc64: bad arguments");
}

int nmpc_ls_prepare(double *G, int32_t n, int32_t ld, int64_t stride_g, double ridge_rel,
                    double *X, int64_t stride_x, int32_t groups, void *stream)
{
    if (!G || !X || n < 1 || ld < n || groups < 1 || groups > 65535 || ridge_rel < 0 ||
        (groups > 1 && (stride_g < (int64_t)n * ld || stride_x < (int64_t)n * ld)))
        return net_fail(NMPC_E_ARG, "ls_prepare: bad arguments");
    long long sg = stride_g, sx = stride_x;
    void *args[] = {(void *)&G, (void *)&n, (void *)&ld, (void *)&sg, (void *)&ridge_rel,
                    (void *)&X, (void *)&sx};
    NET_TRY(hipLaunchKernel(nmpc::ls_prepare_kernel(), dim3(groups), dim3(1024), args, 0,
                            (hipStream_t)stream));
    return NMPC_OK;
}

int nmpc_net_features(const double *x0, const double *xref, int32_t count, int32_t ns,
                      int32_t lattice, int32_t win, int32_t planes, float *Xf, uint16_t *Xb,
                      int32_t ld, void *stream)
{
    if (!x0 || !xref || (!Xf && !Xb) || count < 1 || ns < 1 || lattice < 1 || ns % lattice ||
        win < ns / lattice || (win - ns / lattice) % 2 || (planes != 2 && planes != 5))
        return net_fail(NMPC_E_ARG, "features: bad arguments");
    if (ld < planes * win * win + lattice * lattice)
        return net_fail(NMPC_E_ARG, "features: ld too small");
    nmpc::FeatArgs a{x0, xref, count, ns, lattice, win, planes, ld, Xf, Xb};
    void *args[] = {(void *)&a};
    NET_TRY(hipLaunchKernel(nmpc::features_kernel(), dim3(count * lattice * lattice), dim3(256),
                            args, 0, (hipStream_t)stream));
    return NMPC_OK;
}

int nmpc_relu_grad(float *dh, const float *h, uint16_t *dhb, int64_t n, void *stream)
{
    if (!dh || !h || !dhb || n < 0) return net_fail(NMPC_E_ARG, "relu_grad: bad arguments");
    long long nn = n;
    void *args[] = {(void *)&dh, (void *)&h, (void *)&dhb, (void *)&nn};
    NET_TRY(hipLaunchKernel(nmpc::relu_grad_kernel(), dim3(grid_for((size_t)n)), dim3(256), args,
                            0, (hipStream_t)stream));
    return NMPC_OK;
}

int nmpc_colsum(const float *A, int32_t M, int32_t N, int32_t lda, float *out, void *stream)
{
    if (!A || !out || M < 1 || N < 1 || lda < N) return net_fail(NMPC_E_ARG, "colsum: bad arguments");
    void *args[] = {(void *)&A, (void *)&M, (void *)&N, (void *)&lda, (void *)&out};
    NET_TRY(hipLaunchKernel(nmpc::colsum_kernel(), dim3((N + 255) / 256), dim3(256), args, 0,
                            (hipStream_t)stream));
    return NMPC_OK;
}

int nmpc_mse_grad(const float *Y, int32_t ldy, const float *T, int32_t ldt, int32_t M, int32_t N,
                  float scale, float *dY, uint16_t *dYb, int32_t lddy, float *row_sse, void *stream)
{
    if (!Y || !T || !dY || !dYb || !row_sse || M < 1 || N < 1 || ldy < N || ldt < N || lddy < N)
        return net_fail(NMPC_E_ARG, "mse_grad: bad arguments");
    void *args[] = {(void *)&Y, (void *)&ldy, (void *)&T, (void *)&ldt, (void *)&M, (void *)&N,
                    (void *)&scale, (void *)&dY, (void *)&dYb, (void *)&lddy, (void *)&row_sse};
    NET_TRY(hipLaunchKernel(nmpc::mse_kernel(), dim3((M + 255) / 256), dim3(256), args, 0,
                            (hipStream_t)stream));
    return NMPC_OK;
}

int nmpc_adam(float *w, const float *g, float *m, float *v, uint16_t *wb, int64_t n, float lr,
              float beta1, float beta2, float eps, float weight_decay, int32_t step, void *stream)
{
    if (!w || !g || !m || !v || n < 1 || step < 1) return net_fail(NMPC_E_ARG, "adam: bad arguments");
    nmpc::AdamArgs a{w, g, m, v, wb, (long long)n, lr, beta1, beta2, eps, weight_decay, step};
    void *args[] = {(void *)&a};
    NET_TRY(hipLaunchKernel(nmpc::adam_kernel(), dim3(grid_for((size_t)n)), dim3(256), args, 0,
                            (hipStream_t)stream));
    return NMPC_OK;
}

int nmpc_to_bf16(const float *x, uint16_t *y, int64_t n, void *stream)
{
    if (!x || !y || n < 0) return net_fail(NMPC_E_ARG, "to_bf16: bad arguments");
    long long nn = n;
    void *args[] = {(void *)&x, (void *)&y, (void *)&nn};
    NET_TRY(hipLaunchKernel(nmpc::to_bf16_kernel(), dim3(grid_for((size_t)n)), dim3(256), args, 0,
                            (hipStream_t)stream));
    return NMPC_OK;
}

int nmpc_pack_inputs(const double *u, int32_t count, int32_t N, int32_t m, float scale, float *rows,
                     int32_t ldr, void *stream)
{
    if (!u || !rows || count < 1 || N < 1 || m < 1 || ldr < N) return net_fail(NMPC_E_ARG, "pack: bad arguments");
    void *args[] = {(void *)&u, (void *)&count, (void *)&N, (void *)&m, (void *)&scale,
                    (void *)&rows, (void *)&ldr};
    NET_TRY(hipLaunchKernel(nmpc::pack_u_kernel(), dim3(grid_for((size_t)count * N * m)), dim3(256),
                            args, 0, (hipStream_t)stream));
    return NMPC_OK;
}

int nmpc_unpack_inputs(const float *rows, int32_t ldr, int32_t count, int32_t N, int32_t m,
                       float scale, double *u, void *stream)
{
    if (!u || !rows || count < 1 || N < 1 || m < 1 || ldr < N) return net_fail(NMPC_E_ARG, "unpack: bad arguments");
    void *args[] = {(void *)&rows, (void *)&ldr, (void *)&count, (void *)&N, (void *)&m,
                    (void *)&scale, (void *)&u};
    NET_TRY(hipLaunchKernel(nmpc::unpack_u_kernel(), dim3(grid_for((size_t)count * N * m)),
                            dim3(256), args, 0, (hipStream_t)stream));
    return NMPC_OK;
}

}  // extern "C"
