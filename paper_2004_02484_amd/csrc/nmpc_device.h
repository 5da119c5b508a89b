// nmpc_device.h -- argument blocks shared by the HIP kernels and the host
// runtime of the double-layer Jacobi NMPC library (internal header).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace nmpc {

constexpr int kWave = 64;       // CDNA wavefront width
constexpr int kMaxWaves = 16;   // waves per workgroup (1024 threads)
constexpr int kMaxM = 64;       // inputs per stage
constexpr int kMaxLy = 8;       // input lattice rows
constexpr int kMaxCx = 6;       // columns per lane: nsx <= 16 * 6 = 96
constexpr int kMaxLx = 8;       // input lattice columns
constexpr size_t kLdsBytes = 160 * 1024;   // LDS of a gfx950 CU (one workgroup's limit)

constexpr int kActive = -1;
constexpr int kStatusOk = 0;        // == NMPC_OK
constexpr int kStatusNoconv = 2;    // == NMPC_E_NOCONV
constexpr int kStatusNonfinite = 3; // == NMPC_E_NONFINITE

// Instance modes; kModeFp32 / kModeFp64 double as kernel precision tags.
constexpr int kModeFp64 = 0;
constexpr int kModeFp32 = 1;
constexpr int kModeFp64Redo = 2;   // FP32 test passed: redo that iterate in FP64

// Upper-layer splittings (values of nmpc_options.upper).
constexpr int kUpperJacobi = 0;
constexpr int kUpperFgs = 1;
constexpr int kUpperBgs = 2;
constexpr int kUpperSgs = 3;

struct DevProblem {
    int nsx, nsy, n, N, m, lx, ly;   // n: padded points per stage, nsy * 16 * CX
    double h, k0, k1, q, r, gamma;
    double tau, ulo, uhi;            // input box by log barrier (tau = 0: none)
    double idx2, idy2, c0;   // 1/dx^2, 1/dy^2 (0 in 1D), 2/dx^2 + 2/dy^2
};

// Per-instance iteration state; two copies, indexed by kernel parity.
struct InstState {
    int status;   // kActive or a final status
    int mode;     // kModeFp32, kModeFp64 or kModeFp64Redo
    int e;        // evaluations done (residual slot of evaluation e is e % 3)
    int j;        // index of the last evaluated iterate S^j
    int pending;  // 1: an FP64 correction step is still owed
    int f32;      // evaluations run with FP32 sweeps
    int eonly;    // 1: the last evaluation stopped after the residual (no S^{j+1})
    int pad;
};

struct IterArgs {
    DevProblem P;
    const double *gx, *gy;          // [lx][nsx], [ly][nsy]
    const double *x0;               // [B][n]
    const double *xref;             // [B][...]
    long long xref_inst_stride;     // elements between instances
    int xref_stage_stride;          // 0 or n
    double *X[2], *U[2], *LAM[2];   // trajectory double buffer [B][N][n] / [B][N][m]
    unsigned long long *rst;        // [3][B][N] per-stage r_scaled bit patterns
    unsigned long long *pst;        // [3][B][N] per-stage r_paper bit patterns
    InstState *st;                  // [2][B]
    int *iters;                     // [B] index of the returned iterate
    double *rfin;                   // [B][2] residuals of the returned iterate
    int *ctr;                       // [0] kernel base index, [2] finished, [3] in FP32 phase
    int kofs;                       // this launch's index within a captured sequence
    int B, units, per_xcd;
    long long rslot;                // residual slot stride of rst / pst
    double tol;
    int max_iter, n_sw, n_schur;
    int n_sw_lam;                   // rollout: costate sweeps per stage (n_sw: state sweeps)
    int residual_only, res_slot;
    int res_first_stage;            // residual_only: unit b evaluates stage 0 of instance b only
    int gs_pf;                      // Gauss-Seidel kernel: LDS holds a stage prefetch region
    int xp_lds;                     // Jacobi kernel: x_{i-1} is copied into LDS (after the
                                    // layout's total) while the stage's first stencils run
    int eval_fp64;                  // FP32 kernel: also takes the FP64 phase's owed
                                    // evaluation-only units (residual in FP64, no step)
    double omega;                   // Gauss-Seidel kernel: over-relaxation of each stage's step
    int fp32_finish;                // FP32 phase: a passed test finishes (no FP64 correction)
    double *apart;                  // input box: [B][N] step limit of each stage's update
    int *aupd;                      // input box: [B] 1 + launch index of the instance's last update
    int res_paper;                  // the test is on r_paper (|K|_inf) instead of r_scaled
    unsigned long long *du;         // [B][2] FP64 correction step of an FP32-sweep solve: max |du|,
                                    // max |u^{j+1}| (bit patterns of non-negative doubles)
};

struct InitArgs {
    int count, B, N, nsx, nsy, sx, m, mode;
    int trajectory_only;            // 1: write S^0 only, keep the iteration state
    int nst;                        // stages written per instance (0: all N)
    int pad_only;                   // 1: of x and lambda write only the zero padding (the
                                    // start's rollout writes the grid points)
    int project;                    // 1: move given inputs strictly inside [ulo, uhi]
    double ulo, uhi;                // input box (with project)
    const double *x0, *wx, *wu, *wl;
    double *X, *U, *LAM;
    InstState *st;
    int *iters, *ctr;
    unsigned long long *du;         // [B][2] zeroed with the iteration state
};

struct OutArgs {
    int count, N, nsx, nsy, sx, m;
    int vec;                        // 1: column pairs as 16-byte accesses (nsx, sx even,
                                    // ox and ol 16-byte aligned)
    const int *iters;
    const double *X[2], *U[2], *LAM[2];
    double *ox, *ou, *ol;
};

// One problem class of a ragged batch, as the ragged kernel sees it.
struct RgClass {
    DevProblem P;             // P.n = nsy * 16 * cx (padded points per stage)
    const double *gx, *gy;    // [lx][nsx], [ly][nsy]
    int tile;                 // tile case of the ragged kernel: 3 * (cx case) + ry - 1
    int sx;                   // padded row stride 16 * cx
};

// Per-instance layout of a ragged batch (device arrays, instance order).
struct RgArgs {
    const RgClass *cls;       // [classes]
    const int *icls;          // class of each instance
    const long long *xoff;    // padded x0 / xref offset (one stage)
    const long long *soff;    // padded X / LAM trajectory offset
    const long long *uoff;    // U trajectory offset (dense == padded)
    const long long *dxoff;   // dense x0 / xref offset
    const long long *dsoff;   // dense X / LAM trajectory offset
    const long long *ustart;  // first stage-residual index (sum of earlier horizons)
    const int2 *umap;         // per unit of the launch's tile case: (instance, stage);
                              // instance < 0: no work
    int count;
};

// Streaming (multi-pass) Jacobi iteration for grids beyond one workgroup:
// dense stage layout, one workgroup per (instance, stage, grid row).
struct StreamArgs {
    DevProblem P;                   // P.n unused (dense: nsx * nsy)
    const double *gx, *gy;          // [lx][nsx], [ly][nsy]
    const double *x0, *xref;        // dense [B][n], xref as in IterArgs
    long long xref_inst_stride;
    int xref_stage_stride;
    double *X[2], *U[2], *LAM[2];   // [B][N][n] / [B][N][m]
    // per-point scratch [B][N][n], each in double slots (T values at the front)
    double *b1, *b2, *invd, *cpk, *g2, *y5, *ytmp, *y4, *y4tmp, *cp;
    double *sc;                     // [B][N][ly][nsx] column sums of B v
    double *kun, *v3;               // [B][N][m]
    double *rowt;                   // [B][N][nsy][kMaxLx] row partials of B^T y4 (multi-pass)
    unsigned long long *rst, *pst;  // [B][N] stage norms (bit patterns)
    double *part;                   // [B][N][units per stage][kMaxM] partial B^T lambda / y4
    double *part2;                  // the same, B^T y4 of the first Schur step when the
                                    // residual pass takes that step
    unsigned long long *unorm;      // [B][N][units per stage][2] partial max |K^x|, |K^lambda|
    int nstrip, nrb;                // lower pass: column strips and row blocks per stage
    long long lunits;               // lower pass: count * N * nrb * nstrip wave units
    int lper_xcd;                   // lower pass: workgroups per XCD run
    InstState *st;                  // [B]
    int *work;                      // [B] 1: the instance takes a step in this iteration,
                                    // 2: that step is the FP64 correction of an FP32-sweep solve
    unsigned long long *du;         // [B][2] as IterArgs::du
    int res_paper;                  // the test is on r_paper instead of r_scaled
    double *apart;                  // input box: [B][N] step limit of each stage
    int *iters;
    double *rfin;
    int *ctr;                       // [2] finished, [3] in the FP32 phase
    long long units;                // count * N * ceil(nsy / kStreamRows) row blocks
    int per_xcd, count;
    double tol;
    int max_iter, n_sw, n_schur;
};

// Grid rows per workgroup of the streaming passes; a pass stages `arrays`
// arrays of (kStreamRows + 2) rows of elem-byte values in LDS (at most two of
// 8 bytes).
constexpr int kStreamRows = 8;
__host__ __device__ inline size_t stream_lds_bytes(int nsx, int elem = 8, int arrays = 2)
{
    return (size_t)arrays * (kStreamRows + 2) * nsx * elem;
}

// The marching-strip passes (two point-Jacobi sweeps per solve): one wave per
// strip of kLowerCols owned grid columns (64 lanes = the strip and kLowerHaloX
// halo columns each side: the residual pass fused with the first Schur step
// needs four) and kLowerRows grid rows, marching down the rows from kLowerHalo
// rows above the block (kLowerRows + 6 a multiple of the lower pass's
// prefetch distance, 6).
constexpr int kLowerRows = 30;
constexpr int kLowerHalo = 3;
constexpr int kLowerHaloX = 4;
constexpr int kLowerCols = kWave - 2 * kLowerHaloX;

struct StreamKernels {
    const void *bsep, *res, *stage, *decide, *jf, *axx, *jft, *v3, *advance;
    const void *lower, *lower_fin;         // fused Schur step, final block (v3 from partials)
    const void *res1;                      // residual pass with the first Schur step
    const void *box_lim, *box_apply;       // input box: stage limits, then the cut step
};
StreamKernels stream_kernels(int prec);

// Explicit-Euler plant step of a batch (closed-loop simulation).
struct PlantArgs {
    long long count;
    int nsx, nsy, lx, ly, ldu;   // ldu: elements between instances' inputs
    const double *x, *u, *gx, *gy;
    double *out;
    double dt, k0, k1, idx2, idy2;
};

// Tile configuration of one iteration-kernel instance.
struct TileCfg {
    int cx, rows, max_waves;
};

// Byte offsets into a workgroup's dynamic LDS.
struct LdsOff {
    size_t edge, gx, gy, gxf, gyf, uvec, v3, kun, red, nrm, total;
};

// Gauss-Seidel stage prefetch: x_i and lambda_i of the next stage (n padded
// points each) copied into LDS while the current stage runs, in 1 KB chunks
// (64 lanes x 16 bytes); doubles per array region, after the layout's total.
__host__ __device__ inline size_t gs_pf_doubles(int n) { return (size_t)((n * 8 + 1023) / 1024) * 128; }
__host__ __device__ inline size_t gs_pf_bytes(int n) { return 2 * gs_pf_doubles(n) * 8; }
// Jacobi kernel: one such array (x_{i-1}).
__host__ __device__ inline size_t xp_stage_bytes(int n) { return gs_pf_doubles(n) * 8; }

__host__ __device__ inline size_t lds_align16(size_t p) { return (p + 15) & ~(size_t)15; }

// GT tile rows (16-lane groups) per workgroup, W waves, CX columns and RY rows
// per lane, tsize bytes per sweep value, LX x LY input lattice.
__host__ __device__ inline LdsOff lds_layout(int GT, int W, int CX, int tsize, int LX, int LY,
                                             int RY)
{
    LdsOff o;
    size_t p = 0;
    // edges hold FP64 values for the residual stencils and T values later
    o.edge = p; p = lds_align16(p + (size_t)2 * 2 * GT * 16 * CX * (tsize > 8 ? tsize : 8));
    o.gx = p;   p = lds_align16(p + (size_t)LX * 16 * CX * 8);
    o.gy = p;   p = lds_align16(p + (size_t)LY * GT * RY * 8);
    o.gxf = p;  p = lds_align16(p + (size_t)LX * 16 * CX * 4);
    o.gyf = p;  p = lds_align16(p + (size_t)LY * GT * RY * 4);
    o.uvec = p; p = lds_align16(p + (size_t)kMaxM * 8);
    o.v3 = p;   p = lds_align16(p + (size_t)kMaxM * 8);
    o.kun = p;  p = lds_align16(p + (size_t)kMaxM * 8);
    o.red = p;  p = lds_align16(p + (size_t)W * kMaxM * 8);
    o.nrm = p;  p = lds_align16(p + (size_t)W * 4 * 8);
    o.total = p;
    return o;
}

// nmpc_info.err_vs_fp64 of one result from its final state and the recorded
// FP64 correction step (host code, nmpc_runtime.hip).
double fp32_step_error(bool fp32, bool finish, const InstState &s, const unsigned long long *du);
int eval_only_visits(bool fp32, bool finish, bool streaming, const InstState &s);

// ry = 0 selects the default tile height for (prec, cx).
const void *iterate_kernel(int prec, int cx, int ry, int lx, int ly, TileCfg *cfg);
// Gauss-Seidel kernel (one workgroup per instance); arguments (IterArgs, int upper).
const void *gs_kernel(int prec, int cx, int ry, int lx, int ly, TileCfg *cfg);
const void *init_kernel();
const void *box_apply_kernel();   // (IterArgs): input-box step rule after an iteration launch
const void *choose_flags_kernel();
const void *choose_copy_kernel();
const void *rollout_kernel(int cx, int lx, int ly, TileCfg *cfg);
const void *pad_kernel();
const void *advance_kernel();
const void *output_kernel();

// One instance's results gathered on the device, so that the host reads a
// batch's results with one copy: both state slots, the final norms, the
// FP64 correction step, the iteration count and the start used.
struct InfoPack {
    InstState s[2];
    double rf[2];
    unsigned long long du[2];
    int iters, used;
};
struct PackArgs {
    const InstState *st;            // [2][B]
    const int *iters;
    const double *rfin;             // [B][2]
    const unsigned long long *du;   // [B][2]
    const int *start;               // [B] or null
    int count, B;
    InfoPack *out;                  // [count]
};
const void *info_pack_kernel();     // (PackArgs)

const void *shift_kernel();   // (const double *s, double *out, long long count, int N, long long w)
const void *plant_kernel();   // (PlantArgs)

// Ragged batch kernels (4 x 4 input lattice); waves: 8, 12 or 16; tcase: the
// tile case of ragged_tile (nullptr where the case is not built).
const void *ragged_iterate_kernel(int prec, int waves, int tcase);
const void *ragged_pad_kernel();
const void *ragged_init_kernel();
const void *ragged_output_kernel();
const void *ragged_box_apply_kernel();   // (IterArgs, RgArgs): input-box step rule of one case
// tile case of a class for a launch of `waves` waves, or -1
int ragged_tile(int nsx, int nsy, int waves, int *cx, int *ry);

}  // namespace nmpc
