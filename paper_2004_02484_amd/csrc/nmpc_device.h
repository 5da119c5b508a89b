// nmpc_device.h -- argument blocks shared by the HIP kernels and the host
// runtime of the double-layer Jacobi NMPC library (internal header).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace nmpc {

constexpr int kWave = 64;       // CDNA wavefront width
constexpr int kMaxWaves = 16;   // waves per workgroup (1024 threads)
constexpr int kMaxRows = 64;    // rows per stage held by one workgroup
constexpr int kMaxLy = 8;       // input lattice rows
constexpr int kMaxM = 64;       // inputs per stage

constexpr int kActive = -1;
constexpr int kStatusOk = 0;        // == NMPC_OK
constexpr int kStatusNoconv = 2;    // == NMPC_E_NOCONV
constexpr int kStatusNonfinite = 3; // == NMPC_E_NONFINITE

struct DevProblem {
    int nsx, nsy, n, N, m, lx, ly;
    double h, k0, k1, q, r, gamma;
    double idx2, idy2, c0;   // 1/dx^2, 1/dy^2 (0 in 1D), 2/dx^2 + 2/dy^2
};

// Per-instance iteration state; two copies, indexed by kernel parity.
struct InstState {
    int status;   // kActive or a final status
    int mode;     // 1: lower layer in FP32, 0: FP64
    int off;      // iterate index j = kernel index - off
    int pending;  // 1: an FP64 correction step is still owed
    int f32;      // iterations run with FP32 sweeps
    int pad[3];
};

struct IterArgs {
    DevProblem P;
    const double *gx, *gy;          // [lx][nsx], [ly][nsy]
    const double *x0;               // [B][n]
    const double *xref;             // [B][...]
    long long xref_inst_stride;     // elements between instances
    int xref_stage_stride;          // 0 or n
    double *X[2], *U[2], *LAM[2];   // trajectory double buffer [B][N][n] / [B][N][m]
    unsigned long long *racc;       // [3][B] r_scaled bit patterns
    unsigned long long *pacc;       // [3][B] r_paper bit patterns
    InstState *st;                  // [2][B]
    int *iters;                     // [B] index of the returned iterate
    double *rfin;                   // [B][2] residuals of the returned iterate
    int *ctr;                       // [0] kernel index, [2] finished instances
    unsigned *wgdone;               // workgroups finished in the current kernel
    unsigned long long *work_units; // (instance, stage) units evaluated
    int B, units, per_xcd;
    double tol;
    int max_iter, n_sw, n_schur;
    int residual_only;
};

struct InitArgs {
    int count, B, N, n, m, mode;
    const double *x0, *wx, *wu, *wl;
    double *X, *U, *LAM;
    InstState *st;
    unsigned long long *racc, *pacc;
    int *iters, *ctr;
    unsigned *wgdone;
};

struct OutArgs {
    int count, N, n, m;
    const int *iters;
    const double *X[2], *U[2], *LAM[2];
    double *ox, *ou, *ol;
};

const void *iterate_kernel(int prec, int rows, int lx, int ly);
const void *init_kernel();
const void *output_kernel();

}  // namespace nmpc
