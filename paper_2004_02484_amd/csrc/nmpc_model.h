// nmpc_model.h -- argument block of the model engine (internal header): the
// double-layer method for further members of the paper's PDE class (Sec. 2)
// on grids of up to kModelMaxNodes nodes, one workgroup per instance.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nmpc {

constexpr int kModelHeat = 0;    // w_t = k0 (1 + k1 w) Lap w + B u (dense B)
constexpr int kModelPlate = 1;   // w_t = alpha Lap w - beta (w - Ta) - rad (w^4 - Ta^4), inputs = node values
constexpr int kModelWave = 2;    // W_tt + damp W_t = k0 (1 + k1 W) Lap W + B u, state (W, W_t)

constexpr int kModelMaxNodes = 4096;
constexpr int kModelMaxM = 64;
constexpr int kModelMaxN = 256;

struct ModelArgs {
    int model, neumann, nsx, nsy, nodes;
    int nxg;          // state entries per stage in the grid layout: nodes (plate: actuator
                      // entries unused), or 2 nodes (wave: W then W_t)
    int m, N;
    double h, q, qv, r, gamma, tau, ulo, uhi;
    double alpha, beta, rad, tamb, k0, k1, damp;
    double idx2, idy2, lpp;    // 1/dx^2, 1/dy^2 (0 in 1D), diagonal of the Laplacian
    const int *nodeinp;        // [nodes] plate: input index of an actuator node, -1 for a state
    const int *act;            // [m] plate: node of each input
    const double *B;           // [nodes][m] heat / wave
    const double *x0;          // [count][nxg]
    const double *xref;        // [count][nodes] (plate: the actuator entries are u_ref)
    double *X[2], *U[2], *LAM[2];   // [count][N][nxg], [count][N][m], [count][N][nxg]
    double *lim;               // [count][N] fraction-to-the-boundary limit of each stage's step
    int *info_i;               // [count][4]: iterations, status, buffer of the returned
                               // iterate, stage passes run
    double *info_d;            // [count][2]: r_scaled, r_paper of the returned iterate
    int count;
    double tol;
    int max_iter, n_sw, n_schur, upper, res_paper;
    int residual_only;         // evaluate the norms of the iterate in buffer 0 only
    double *out_x, *out_u, *out_lam;   // dense outputs (may be null)
};

// S^0 into buffer 0: cold (x_i = x0, u_i = u_cold, lambda_i = 0) or the given
// dense start; inputs clipped strictly inside an input box; the plate's
// actuator entries of x and lambda are zero. Arguments (ModelArgs, ModelInit).
struct ModelInit {
    const double *wx, *wu, *wl;
    double u_cold;
    int project;
};

const void *model_kernel(int model, int ppt);
const void *model_init_kernel();

}  // namespace nmpc
