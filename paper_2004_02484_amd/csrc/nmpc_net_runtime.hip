// nmpc_net_runtime.hip -- C ABI of the warm-start network kernels: argument
// checks and launches on the caller's stream (all pointers are device memory).
#include <hip/hip_runtime.h>

#include <algorithm>
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

}  // namespace

extern "C" {

int nmpc_gemm_bf16(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K,
                   const uint16_t *A, int32_t lda, const uint16_t *B, int32_t ldb, float beta,
                   float *C, int32_t ldc, const float *bias, int32_t relu, uint16_t *Cb,
                   int32_t ldcb, void *stream)
{
    if (M < 1 || N < 1 || K < 1 || !A || !B || (!C && !Cb))
        return net_fail(NMPC_E_ARG, "gemm: bad sizes or NULL operand");
    if (lda < (trans_a ? M : K) || ldb < (trans_b ? K : N) || (C && ldc < N) || (Cb && ldcb < N))
        return net_fail(NMPC_E_ARG, "gemm: leading dimension too small");
    if (beta != 0.f && !C) return net_fail(NMPC_E_ARG, "gemm: beta needs C");
    nmpc::GemmArgs g{M, N, K, A, lda, B, ldb, beta, C, ldc, bias, relu ? 1 : 0, Cb, ldcb};
    void *args[] = {(void *)&g};
    NET_TRY(hipLaunchKernel(nmpc::gemm_kernel(trans_a != 0, trans_b != 0),
                            dim3((N + 63) / 64, (M + 63) / 64), dim3(256), args, 0,
                            (hipStream_t)stream));
    return NMPC_OK;
}

int nmpc_net_windows(const double *x0, const double *xref, int32_t count, int32_t ns,
                     int32_t lattice, int32_t win, uint16_t *out, uint16_t *out_lo, int32_t ld,
                     void *stream)
{
    if (!x0 || !xref || !out || count < 1 || ns < 1 || lattice < 1 || ns % lattice || win < 1)
        return net_fail(NMPC_E_ARG, "windows: bad arguments");
    if (ld < 2 * win * win + lattice * lattice) return net_fail(NMPC_E_ARG, "windows: ld too small");
    nmpc::WinArgs a{x0, xref, count, ns, lattice, win, ld, out, out_lo};
    void *args[] = {(void *)&a};
    NET_TRY(hipLaunchKernel(nmpc::windows_kernel(),
                            dim3(grid_for((size_t)count * lattice * lattice * ld)), dim3(256),
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

int nmpc_split_bf16(const float *x, uint16_t *hi, uint16_t *lo, int64_t n, void *stream)
{
    if (!x || !hi || !lo || n < 0) return net_fail(NMPC_E_ARG, "split_bf16: bad arguments");
    long long nn = n;
    void *args[] = {(void *)&x, (void *)&hi, (void *)&lo, (void *)&nn};
    NET_TRY(hipLaunchKernel(nmpc::split_bf16_kernel(), dim3(grid_for((size_t)n)), dim3(256), args,
                            0, (hipStream_t)stream));
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
