// nmpc_net.h -- argument blocks of the warm-start network kernels (internal).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace nmpc {

struct GemmArgs {
    int M, N, K;
    const unsigned short *A;   // bf16
    int lda;
    const unsigned short *B;   // bf16
    int ldb;
    float beta;
    float *C;                  // fp32 output (may be null)
    int ldc;
    const float *bias;         // [N] or null
    int relu;
    unsigned short *Cb;        // bf16 output (may be null)
    int ldcb;
    int ksplit, kc;            // K split in ksplit parts of kc (blockIdx.z = part); > 1:
    float *work;               // raw partial products [ksplit][M][N], the epilogue in
                               // k_gemm_reduce
};

struct GemmMxArgs {
    int M, N, K;
    const void *A;             // float or double (kernel's input type)
    int lda;
    const void *B;
    int ldb;
    double alpha, beta;
    const void *Cin;           // beta term (null: C itself); accumulator type
    void *C;                   // accumulator type (float or double)
    int ldc;
    long long sa, sb, sc;      // element offsets between groups
    int ksplit, kc;            // K split in ksplit parts of kc (blockIdx.z = group * ksplit + part)
    void *work;                // ksplit > 1: partial sums [groups][ksplit][M][N]
};

struct FeatArgs {
    const double *x0, *xref;   // [count][ns * ns]
    int count, ns, L, win, planes, ld;
    float *Xf;                 // [count * L * L][ld] fp32 (may be null)
    unsigned short *Xb;        // [count * L * L][ld] bf16 (may be null)
};

// The per-actuator map of the forward pass fused with the feature gather
// (k_map_fwd): partial sums over K parts of Y[b][p] = X(b, p) Ws[p].
struct MapArgs {
    const double *x0, *xref;   // [count][ns * ns]
    int count, ns, L, win, planes;
    const float *Ws;           // [L * L][K0][N]
    int K0, N;
    int chunks, cpp, ksplit;   // 32-pixel window chunks, chunks per part, parts
    float *work;               // [L * L][ksplit][count][N]
};

struct AdamArgs {
    float *w;
    const float *g;
    float *m, *v;
    unsigned short *wb;        // bf16 copy (may be null)
    long long n;
    float lr, b1, b2, eps, wd;
    int step;
};

const void *gemm_kernel(int ta, int tb);
const void *gemm_mx_kernel(int ta, int in64, int acc64);
const void *ls_prepare_kernel();
const void *splitk_reduce_kernel();
const void *gemm_reduce_kernel();   // (GemmArgs): split-K sum and the bf16 GEMM's epilogue
// The bf16 GEMM with K split in `ksplit` parts (work: ksplit * M * N floats),
// for the network object; ksplit = 1 is nmpc_gemm_bf16.
int gemm_bf16_split(int ta, int tb, int M, int N, int K, const uint16_t *A, int lda, const uint16_t *B,
                    int ldb, float beta, float *C, int ldc, const float *bias, int relu, uint16_t *Cb,
                    int ldcb, int ksplit, float *work, void *stream);
const void *features_kernel();
const void *map_fwd_kernel();
// Y rows b L^2 + p (row stride L^2 N) = beta Y + X(b, p) Ws[p] for count
// instances, the features gathered inside the product (work: 8 L^2 count N
// floats); fused form of nmpc_net_features followed by the grouped fp32 map.
int map_forward(const double *x0, const double *xref, int count, int ns, int L, int win, int planes,
                const float *Ws, int K0, int N, float beta, float *Y, float *work, void *stream);
const void *relu_grad_kernel();
const void *colsum_kernel();
const void *mse_kernel();
const void *adam_kernel();
const void *to_bf16_kernel();
const void *pack_u_kernel();
const void *unpack_u_kernel();

}  // namespace nmpc
