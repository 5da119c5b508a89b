// nmpc_runtime.hip -- host runtime and C ABI of the double-layer Jacobi NMPC
// library: validation, device workspace, the upper-iteration launch loop
// (replayed as a captured hipGraph of check_every launches), convergence
// polling and result copies.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "nmpc.h"
#include "nmpc_device.h"

using nmpc::InitArgs;
using nmpc::InstState;
using nmpc::IterArgs;
using nmpc::OutArgs;
using nmpc::TileCfg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(e_ == hipErrorOutOfMemory ? NMPC_E_OOM : NMPC_E_DEVICE,       \
                        std::string(#expr) + ": " + hipGetErrorString(e_));           \
    } while (0)

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

struct nmpc_handle {
    nmpc_problem prob{};
    nmpc_options opt{};
    int max_batch = 0;
    int n = 0, m = 0, N = 0;
    int sx = 0, np = 0;                    // padded row stride (16 * CX), padded points per stage
    struct Kern {
        const void *fn = nullptr;
        TileCfg cfg{};
        int waves = 0;
        size_t lds = 0;
        int pf = 0;                        // Gauss-Seidel: stage prefetch region in LDS
    } kern[2];                             // [kModeFp64], [kModeFp32]
    Kern gs[2];                            // Gauss-Seidel kernels (upper != Jacobi)
    bool streaming = false;                // multi-pass kernels (grids beyond one workgroup)
    double *d_stream = nullptr;            // streaming scratch (see stream_args)
    int *d_work = nullptr;                 // [B] streaming: instance steps this iteration
    Kern roll;                             // start built from an input trajectory
    int *d_start = nullptr;                // [B] start used per instance
    double *d_apart = nullptr;             // input box: [B][N] step limits
    int *d_aupd = nullptr;                 // input box: [B] last updating launch + 1
    int last_start_kind = 0;
    bool last_fallback = false;
    std::vector<double> gx, gy;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    // second stream of the fallback check: the cold start is built and
    // evaluated there while the input-built start's rollout runs
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    double *d_gx = nullptr, *d_gy = nullptr;
    double *d_S[2] = {nullptr, nullptr};
    double *d_x0 = nullptr, *d_xref = nullptr, *d_out = nullptr;
    unsigned long long *d_rst = nullptr;   // per-stage residual bits [2][3][B][N]
    InstState *d_st = nullptr;             // [2][B]
    int *d_iters = nullptr;                // [B]
    double *d_rfin = nullptr;              // [B][2]
    unsigned long long *d_du = nullptr;    // [B][2] FP64 correction step (max |du|, max |u|)
    int *d_ctr = nullptr;                  // [4]
    int *h_poll = nullptr;                 // pinned
    nmpc::InfoPack *d_info = nullptr;      // [B] results gathered for one copy
    nmpc::InfoPack *h_info = nullptr;      // [B] pinned
    nmpc_model *dense = nullptr;           // dense-B problems: the model engine's handle
    bool timing = false;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    double kernel_ms = 0.0;
    long long launches = 0;
    long long units = 0;                   // evaluated and updated (instance, stage) units
    long long units_eval = 0;              // evaluation-only units
    // [0], [1]: graphs of the FP32 and FP64 kernels; [2]: the first graph of
    // an FP32-sweep solve sized from the previous solve (ensure_first_graph)
    hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
    int graph_count[3] = {-1, -1, -1}, graph_len[3] = {0, 0, 0};
    int last_iters = -1;                   // largest iteration count of the last solve (-1: none)
    size_t xref_len = 0;                   // padded xref elements per instance (device)

    double *X(int b) const { return d_S[b]; }
    double *L(int b) const { return d_S[b] + (size_t)max_batch * N * np; }
    double *U(int b) const { return d_S[b] + (size_t)2 * max_batch * N * np; }
    size_t xref_dense() const { return (size_t)n * (opt.xref_per_stage ? N : 1); }
};

namespace {

int tile_cx(int nsx)
{
    const int cx = (nsx + 15) / 16;
    return cx == 5 ? 6 : cx;
}

// Pick the iteration kernel of precision `prec` for this grid and lattice:
// the Jacobi kernel (gs = false) or the Gauss-Seidel kernel.
int select_kernel(const nmpc_problem *p, int prec, int ry, nmpc_handle::Kern *k, bool gs = false)
{
    TileCfg cfg{};
    const void *fn = gs ? nmpc::gs_kernel(prec, tile_cx(p->nsx), ry, p->lx, p->ly, &cfg)
                        : nmpc::iterate_kernel(prec, tile_cx(p->nsx), ry, p->lx, p->ly, &cfg);
    if (!fn && ry) return fail(NMPC_E_UNSUPPORTED, "no kernel instance with this tile height");
    if (!fn) return fail(NMPC_E_UNSUPPORTED, "no kernel instance for this grid width / input lattice");
    const int groups = (p->nsy + cfg.rows - 1) / cfg.rows;
    const int waves = (groups + 3) / 4;
    if (waves > cfg.max_waves)
        return fail(NMPC_E_UNSUPPORTED, "grid too tall for the fused stage kernel");
    const size_t lds = nmpc::lds_layout(waves * 4, waves, cfg.cx, prec == nmpc::kModeFp32 ? 4 : 8,
                                        p->lx, p->ly, cfg.rows).total;
    if (lds > nmpc::kLdsBytes)
        return fail(NMPC_E_UNSUPPORTED, "tile needs more LDS than a CU has");
    // the Gauss-Seidel kernel prefetches the next stage into LDS where it fits;
    // the Jacobi kernel copies x_{i-1} into LDS where that still leaves room
    // for the workgroups per CU its registers allow (two of up to four waves,
    // one of eight)
    const int np = p->nsy * 16 * cfg.cx;
    const size_t extra = gs ? nmpc::gs_pf_bytes(np) : nmpc::xp_stage_bytes(np);
    const size_t cap = gs || waves > 4 ? nmpc::kLdsBytes : nmpc::kLdsBytes / 2;
    const int pf = lds + extra <= cap ? 1 : 0;
    if (k) {
        k->fn = fn;
        k->cfg = cfg;
        k->waves = waves;
        k->lds = pf ? lds + extra : lds;
        k->pf = pf;
    }
    return NMPC_OK;
}

int check_problem(const nmpc_problem *p)
{
    if (!p) return fail(NMPC_E_ARG, "problem is NULL");
    if (p->dim != 1 && p->dim != 2) return fail(NMPC_E_ARG, "dim must be 1 or 2");
    if (p->nsx < 1 || p->nsy < 1 || p->horizon < 1 || p->lx < 1 || p->ly < 1)
        return fail(NMPC_E_ARG, "sizes must be positive");
    if (p->dim == 1 && (p->nsy != 1 || p->ly != 1))
        return fail(NMPC_E_ARG, "1D problems need nsy == 1 and ly == 1");
    if (p->b_kind != NMPC_B_KRON && p->b_kind != NMPC_B_DENSE)
        return fail(NMPC_E_ARG, "b_kind must be NMPC_B_KRON or NMPC_B_DENSE");
    if (p->b_kind == NMPC_B_DENSE) {
        if (!p->B) return fail(NMPC_E_ARG, "a dense B is NULL");
        for (long long t = 0; t < (long long)p->nsx * p->nsy * p->lx * p->ly; ++t)
            if (!std::isfinite(p->B[t])) return fail(NMPC_E_ARG, "B not finite");
    } else if (!p->gx || !p->gy) {
        return fail(NMPC_E_ARG, "gx/gy are NULL");
    }
    if (!finite_pos(p->h) || !finite_pos(p->r) || !std::isfinite(p->k0) ||
        !std::isfinite(p->k1) || !std::isfinite(p->q) || p->q < 0.0 ||
        !std::isfinite(p->gamma) || p->gamma < 0.0)
        return fail(NMPC_E_ARG, "need h > 0, r > 0, q >= 0, gamma >= 0, finite k0, k1");
    if (!std::isfinite(p->tau) || p->tau < 0.0)
        return fail(NMPC_E_ARG, "tau must be finite and >= 0");
    if (p->tau > 0.0 && !(std::isfinite(p->u_lo) && std::isfinite(p->u_hi) && p->u_lo < 0.0 &&
                          p->u_hi > 0.0))
        return fail(NMPC_E_ARG, "an input box needs finite u_lo < 0 < u_hi (cold start inside)");
    if (p->b_kind == NMPC_B_DENSE) return NMPC_OK;   // sizes checked by the model engine
    for (long long t = 0; t < (long long)p->lx * p->nsx; ++t)
        if (!std::isfinite(p->gx[t])) return fail(NMPC_E_ARG, "gx not finite");
    for (long long t = 0; t < (long long)p->ly * p->nsy; ++t)
        if (!std::isfinite(p->gy[t])) return fail(NMPC_E_ARG, "gy not finite");
    if (p->ly > nmpc::kMaxLy || p->lx > nmpc::kMaxLx || p->lx * p->ly > nmpc::kMaxM)
        return fail(NMPC_E_UNSUPPORTED, "input lattice larger than 8 x 8");
    return NMPC_OK;
}

// Does the fused stage kernel cover this problem?
int check_fused(const nmpc_problem *p)
{
    if (p->nsx > 16 * nmpc::kMaxCx)
        return fail(NMPC_E_UNSUPPORTED, "fused stage kernel needs nsx <= 96");
    for (int prec : {nmpc::kModeFp64, nmpc::kModeFp32}) {
        const int rc = select_kernel(p, prec, 0, nullptr);
        if (rc) return rc;
    }
    return NMPC_OK;
}

int check_options(const nmpc_options *o)
{
    if (!o) return fail(NMPC_E_ARG, "options are NULL");
    if (!(o->tol >= 0.0) || std::isnan(o->tol)) return fail(NMPC_E_ARG, "tol must be >= 0");
    if (o->max_iter < 0 || o->max_iter > 100000000) return fail(NMPC_E_ARG, "bad max_iter");
    if (o->n_sweep < 1 || o->n_sweep > 16) return fail(NMPC_E_ARG, "n_sweep must be 1..16");
    if (o->n_schur < 0 || o->n_schur > 16) return fail(NMPC_E_ARG, "n_schur must be 0..16");
    if (o->precision != NMPC_FP64 && o->precision != NMPC_FP32_SWEEP)
        return fail(NMPC_E_ARG, "unknown precision");
    if (o->check_every < 1 || o->check_every > 4096) return fail(NMPC_E_ARG, "bad check_every");
    if (o->xref_per_stage != 0 && o->xref_per_stage != 1)
        return fail(NMPC_E_ARG, "xref_per_stage must be 0 or 1");
    if (o->tile_rows < 0 || o->tile_rows > 16) return fail(NMPC_E_ARG, "tile_rows must be 0..16");
    if (o->warm_sweeps < 0 || o->warm_sweeps > 1000) return fail(NMPC_E_ARG, "warm_sweeps must be 0..1000");
    if (o->warm_sweeps_lambda < 0 || o->warm_sweeps_lambda > 1000)
        return fail(NMPC_E_ARG, "warm_sweeps_lambda must be 0..1000");
    if (o->fallback != 0 && o->fallback != 1) return fail(NMPC_E_ARG, "fallback must be 0 or 1");
    if (o->upper < NMPC_UPPER_JACOBI || o->upper > NMPC_UPPER_SGS)
        return fail(NMPC_E_ARG, "unknown upper layer");
    if (o->path < NMPC_PATH_AUTO || o->path > NMPC_PATH_STREAM)
        return fail(NMPC_E_ARG, "unknown kernel path");
    if (!(o->omega > 0.0 && o->omega < 2.0))
        return fail(NMPC_E_ARG, "omega must lie in (0, 2)");
    if (o->upper == NMPC_UPPER_JACOBI && o->omega != 1.0)
        return fail(NMPC_E_ARG, "over-relaxation (omega != 1) needs a Gauss-Seidel upper layer");
    if (o->fp32_finish != 0 && o->fp32_finish != 1) return fail(NMPC_E_ARG, "fp32_finish must be 0 or 1");
    if (o->residual != NMPC_RES_SCALED && o->residual != NMPC_RES_PAPER)
        return fail(NMPC_E_ARG, "residual must be NMPC_RES_SCALED or NMPC_RES_PAPER");
    return NMPC_OK;
}

// Kernel path of a problem under options: 1 streaming, 0 fused, or an error.
int choose_path(const nmpc_problem *p, const nmpc_options *o, bool *streaming)
{
    const int fused = o->path == NMPC_PATH_STREAM ? NMPC_E_UNSUPPORTED : check_fused(p);
    if (o->path == NMPC_PATH_FUSED && fused) return fused;
    *streaming = fused != NMPC_OK;
    if (*streaming && o->upper != NMPC_UPPER_JACOBI)
        return fail(NMPC_E_UNSUPPORTED, "the streaming path runs the Jacobi upper layer only");
    if (*streaming && o->fp32_finish)
        return fail(NMPC_E_UNSUPPORTED, "fp32_finish runs on the fused path");
    if (*streaming && nmpc::stream_lds_bytes(p->nsx) > nmpc::kLdsBytes)
        return fail(NMPC_E_UNSUPPORTED, "grid rows too wide for the streaming path");
    g_err.clear();
    return NMPC_OK;
}

int main_prec(const nmpc_options &o)
{
    return o.precision == NMPC_FP32_SWEEP ? nmpc::kModeFp32 : nmpc::kModeFp64;
}

// Kernels of both precisions for the handle's upper layer (tile_rows applies
// to the main precision), with their LDS limits raised where needed.
int select_all(const nmpc_problem *p, const nmpc_options *o, nmpc_handle::Kern (&jk)[2],
               nmpc_handle::Kern (&gk)[2])
{
    for (int prec : {nmpc::kModeFp64, nmpc::kModeFp32}) {
        const int ry = prec == main_prec(*o) ? o->tile_rows : 0;
        const bool gs = o->upper != NMPC_UPPER_JACOBI;
        // the Jacobi kernel always exists: residual launches (fallback) use it
        int rc = select_kernel(p, prec, gs ? 0 : ry, &jk[prec]);
        if (rc) return rc;
        if (gs) {
            rc = select_kernel(p, prec, ry, &gk[prec], true);
            if (rc) return rc;
        }
    }
    return NMPC_OK;
}

int raise_lds(const nmpc_handle::Kern &k)
{
    if (k.fn && k.lds > 48 * 1024)
        HIP_TRY(hipFuncSetAttribute(k.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)k.lds));
    return NMPC_OK;
}

void release(nmpc_handle *h)
{
    if (!h) return;
    for (int q = 0; q < 3; ++q) {
        if (h->gexec[q]) (void)hipGraphExecDestroy(h->gexec[q]);
        if (h->graph[q]) (void)hipGraphDestroy(h->graph[q]);
    }
    for (void *p : {(void *)h->d_gx, (void *)h->d_gy, (void *)h->d_S[0], (void *)h->d_S[1],
                    (void *)h->d_x0, (void *)h->d_xref, (void *)h->d_out, (void *)h->d_rst,
                    (void *)h->d_st, (void *)h->d_iters, (void *)h->d_rfin, (void *)h->d_ctr,
                    (void *)h->d_start, (void *)h->d_stream, (void *)h->d_work,
                    (void *)h->d_apart, (void *)h->d_aupd, (void *)h->d_du, (void *)h->d_info})
        if (p) (void)hipFree(p);
    if (h->h_poll) (void)hipHostFree(h->h_poll);
    if (h->h_info) (void)hipHostFree(h->h_info);
    if (h->ev) (void)hipEventDestroy(h->ev);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->side) (void)hipStreamDestroy(h->side);
    if (h->t0) (void)hipEventDestroy(h->t0);
    if (h->t1) (void)hipEventDestroy(h->t1);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    if (h->dense) nmpc_model_destroy(h->dense);
    delete h;
}

IterArgs iter_args(const nmpc_handle *h, int count)
{
    IterArgs a{};
    const nmpc_problem &p = h->prob;
    a.P.nsx = p.nsx; a.P.nsy = p.nsy; a.P.n = h->np; a.P.N = h->N; a.P.m = h->m;
    a.P.lx = p.lx; a.P.ly = p.ly;
    a.P.h = p.h; a.P.k0 = p.k0; a.P.k1 = p.k1; a.P.q = p.q; a.P.r = p.r; a.P.gamma = p.gamma;
    a.P.tau = p.tau; a.P.ulo = p.u_lo; a.P.uhi = p.u_hi;
    a.apart = h->d_apart; a.aupd = h->d_aupd;
    const double dx = 1.0 / (p.nsx + 1), dy = 1.0 / (p.nsy + 1);
    a.P.idx2 = 1.0 / (dx * dx);
    a.P.idy2 = p.dim == 2 ? 1.0 / (dy * dy) : 0.0;
    a.P.c0 = 2.0 * a.P.idx2 + 2.0 * a.P.idy2;
    a.gx = h->d_gx; a.gy = h->d_gy;
    a.x0 = h->d_x0; a.xref = h->d_xref;
    a.xref_inst_stride = (long long)h->xref_len;
    a.xref_stage_stride = h->opt.xref_per_stage ? h->np : 0;
    for (int b = 0; b < 2; ++b) { a.X[b] = h->X(b); a.U[b] = h->U(b); a.LAM[b] = h->L(b); }
    a.rst = h->d_rst;
    a.pst = h->d_rst + 3 * (size_t)h->max_batch * h->N;
    a.st = h->d_st; a.iters = h->d_iters; a.rfin = h->d_rfin; a.du = h->d_du;
    a.ctr = h->d_ctr; a.kofs = 0;
    a.B = h->max_batch;
    a.units = count * h->N;
    a.per_xcd = (a.units + 7) / 8;
    a.rslot = (long long)h->max_batch * h->N;
    a.tol = h->opt.tol; a.max_iter = h->opt.max_iter;
    a.n_sw = h->opt.n_sweep; a.n_schur = h->opt.n_schur;
    a.omega = h->opt.omega;
    a.fp32_finish = h->opt.fp32_finish;
    a.res_paper = h->opt.residual == NMPC_RES_PAPER;
    a.residual_only = 0;
    return a;
}

int launch_iterate(nmpc_handle *h, int prec, const IterArgs &a, hipStream_t s)
{
    const nmpc_handle::Kern &k = h->kern[prec];
    IterArgs ak = a;
    ak.xp_lds = k.pf;
    void *args[] = {(void *)&ak};
    HIP_TRY(hipLaunchKernel(k.fn, dim3(8 * a.per_xcd), dim3(nmpc::kWave * k.waves), args, k.lds, s));
    if (h->prob.tau > 0.0 && !a.residual_only)   // input box: step rule of this launch
        HIP_TRY(hipLaunchKernel(nmpc::box_apply_kernel(), dim3(8 * a.per_xcd), dim3(256), args, 0,
                                s));
    return NMPC_OK;
}

// Captured sequence of check_every launches of the precision-`prec` kernel.
// After FP32 sweeps the FP64 phase is the final correction, which takes three
// launches per instance (the FP64 re-evaluation of the accepted iterate with
// the correction step, the evaluation of its result, the final test): its
// graph is four launches long, and the host relaunches it if an instance needs
// more. Its second launch, where the evaluations fall, runs the FP32 kernel
// (two workgroups per CU against one) with eval_fp64 set: it evaluates the
// owed results and leaves every other unit of the FP64 phase to the next
// launch.
int ensure_graph(nmpc_handle *h, int prec, int count)
{
    const int len = (prec == nmpc::kModeFp64 && main_prec(h->opt) == nmpc::kModeFp32)
                        ? std::min(4, h->opt.check_every)
                        : h->opt.check_every;
    if (h->gexec[prec] && h->graph_count[prec] == count && h->graph_len[prec] == len)
        return NMPC_OK;
    if (h->gexec[prec]) { (void)hipGraphExecDestroy(h->gexec[prec]); h->gexec[prec] = nullptr; }
    if (h->graph[prec]) { (void)hipGraphDestroy(h->graph[prec]); h->graph[prec] = nullptr; }
    IterArgs a = iter_args(h, count);
    HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    int rc = NMPC_OK;
    const bool phase64 = prec == nmpc::kModeFp64 && main_prec(h->opt) == nmpc::kModeFp32;
    for (int t = 0; t < len && rc == NMPC_OK; ++t) {
        a.kofs = t;
        a.eval_fp64 = phase64 && t == 1 ? 1 : 0;
        rc = launch_iterate(h, a.eval_fp64 ? nmpc::kModeFp32 : prec, a, h->stream);
    }
    if (rc == NMPC_OK) {
        int *ctr = h->d_ctr;
        void *args[] = {(void *)&ctr, (void *)&len};
        const hipError_t e = hipLaunchKernel(nmpc::advance_kernel(), dim3(1), dim3(64), args, 0,
                                             h->stream);
        if (e != hipSuccess) rc = fail(NMPC_E_DEVICE, std::string("advance: ") + hipGetErrorString(e));
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->stream, &g);
    if (rc != NMPC_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return fail(NMPC_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    h->graph[prec] = g;
    HIP_TRY(hipGraphInstantiate(&h->gexec[prec], g, nullptr, nullptr, 0));
    h->graph_count[prec] = count; h->graph_len[prec] = len;
    return NMPC_OK;
}

// First graph of an FP32-sweep solve whose previous solve converged in J
// iterations: nf = J + 1 FP32 launches (the last one takes the test that
// passes), then the FP64 phase's three launches (the correction step on the
// FP64 kernel, then the evaluation of its result and the final test on the
// FP32 kernel with eval_fp64: a decision needs no FP64 arithmetic, and an
// instance whose final test fails waits for the next FP64 launch). A solve that
// converges as the previous one did ends with this one graph and one poll;
// one that needs more continues with the ordinary graphs (the state machine
// lets each instance wait for the kernel of its phase).
int ensure_first_graph(nmpc_handle *h, int count, int nf)
{
    const int len = nf + 3;
    if (h->gexec[2] && h->graph_count[2] == count && h->graph_len[2] == len) return NMPC_OK;
    if (h->gexec[2]) { (void)hipGraphExecDestroy(h->gexec[2]); h->gexec[2] = nullptr; }
    if (h->graph[2]) { (void)hipGraphDestroy(h->graph[2]); h->graph[2] = nullptr; }
    IterArgs a = iter_args(h, count);
    HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    int rc = NMPC_OK;
    for (int t = 0; t < len && rc == NMPC_OK; ++t) {
        a.kofs = t;
        a.eval_fp64 = t > nf ? 1 : 0;
        const int prec = t == nf ? nmpc::kModeFp64 : nmpc::kModeFp32;
        rc = launch_iterate(h, prec, a, h->stream);
    }
    if (rc == NMPC_OK) {
        int *ctr = h->d_ctr;
        void *args[] = {(void *)&ctr, (void *)&len};
        const hipError_t e = hipLaunchKernel(nmpc::advance_kernel(), dim3(1), dim3(64), args, 0,
                                             h->stream);
        if (e != hipSuccess) rc = fail(NMPC_E_DEVICE, std::string("advance: ") + hipGetErrorString(e));
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->stream, &g);
    if (rc != NMPC_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return fail(NMPC_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    h->graph[2] = g;
    HIP_TRY(hipGraphInstantiate(&h->gexec[2], g, nullptr, nullptr, 0));
    h->graph_count[2] = count; h->graph_len[2] = len;
    return NMPC_OK;
}

int launch_grid(size_t tot) { return (int)std::min<size_t>((tot + 255) / 256 + 1, 8192); }

// Dense device rows [rows][nsx] -> padded rows [rows][sx] in dst.
int pad_rows(nmpc_handle *h, const double *src, double *dst, long long rows)
{
    int nsx = h->prob.nsx, sx = h->sx;
    void *args[] = {(void *)&src, (void *)&dst, (void *)&rows, (void *)&nsx, (void *)&sx};
    HIP_TRY(hipLaunchKernel(nmpc::pad_kernel(), dim3(launch_grid((size_t)rows * sx)), dim3(256),
                            args, 0, h->stream));
    return NMPC_OK;
}

// x0 [count][n] and xref [count][n or N*n] (dense, device) into the handle's
// padded input buffers.
int stage_inputs(nmpc_handle *h, int count, const double *x0, const double *xref)
{
    int rc = pad_rows(h, x0, h->d_x0, (long long)count * h->prob.nsy);
    if (rc) return rc;
    return pad_rows(h, xref, h->d_xref,
                    (long long)count * h->prob.nsy * (h->opt.xref_per_stage ? h->N : 1));
}

enum { kStartCold = 0, kStartGiven = 1, kStartInputs = 2 };

int start_kind(const double *wx, const double *wu, const double *wl)
{
    if (!wx && !wu && !wl) return kStartCold;
    if (wx && wu && wl) return kStartGiven;
    if (!wx && wu) return kStartInputs;
    return -1;
}

int launch_residual(nmpc_handle *h, int count, int buf, int slot, hipStream_t s = nullptr,
                    bool first_stage = false)
{
    IterArgs a = iter_args(h, count);
    a.residual_only = 1;
    a.res_slot = slot;
    if (first_stage) {   // one unit per instance: stage 0
        a.res_first_stage = 1;
        a.units = count;
        a.per_xcd = (count + 7) / 8;
    }
    a.X[0] = h->X(buf); a.U[0] = h->U(buf); a.LAM[0] = h->L(buf);
    return launch_iterate(h, nmpc::kModeFp64, a, s ? s : h->stream);
}

// S^0 for `count` instances in buffer 0 (and the iteration state reset):
// cold, given, or built from an input trajectory; with the fallback option a
// warm start is replaced per instance by the cold one when its residual is
// not smaller.
int build_start(nmpc_handle *h, int count, const double *wx, const double *wu,
                const double *wl)
{
    const int kind = start_kind(wx, wu, wl);
    InitArgs ia{};
    ia.count = count; ia.B = h->max_batch; ia.N = h->N; ia.m = h->m;
    ia.nsx = h->prob.nsx; ia.nsy = h->prob.nsy; ia.sx = h->sx;
    ia.mode = h->opt.precision == NMPC_FP32_SWEEP ? nmpc::kModeFp32 : nmpc::kModeFp64;
    ia.x0 = h->d_x0; ia.wx = wx; ia.wu = wu; ia.wl = wl;
    ia.X = h->X(0); ia.U = h->U(0); ia.LAM = h->L(0);
    ia.st = h->d_st;
    ia.iters = h->d_iters; ia.ctr = h->d_ctr;
    ia.project = h->prob.tau > 0.0 ? 1 : 0;
    ia.du = h->d_du;
    ia.ulo = h->prob.u_lo; ia.uhi = h->prob.u_hi;
    if (h->d_aupd)   // input box: no update recorded for this solve yet (not captured)
        HIP_TRY(hipMemsetAsync(h->d_aupd, 0, sizeof(int) * h->max_batch, h->stream));
    const bool check = kind != kStartCold && h->opt.fallback && !h->streaming;
    // a start built from inputs gets its states and costates from the rollout
    if (kind == kStartInputs && !h->streaming) ia.pad_only = 1;
    {
        void *args[] = {(void *)&ia};
        HIP_TRY(hipLaunchKernel(nmpc::init_kernel(),
                                dim3(launch_grid((size_t)count * h->N * h->np)), dim3(256), args,
                                0, h->stream));
    }
    if (check) HIP_TRY(hipEventRecord(h->ev_fork, h->stream));
    if (h->streaming) {
        if (kind == kStartInputs)
            return fail(NMPC_E_UNSUPPORTED, "the streaming path takes cold or (x, u, lambda) starts");
        h->last_start_kind = kind;
        h->last_fallback = false;
        return NMPC_OK;
    }
    if (kind == kStartInputs) {
        IterArgs a = iter_args(h, count);
        a.units = count;
        a.n_sw = h->opt.warm_sweeps > 0 ? h->opt.warm_sweeps : 24;
        a.n_sw_lam = h->opt.warm_sweeps_lambda > 0 ? h->opt.warm_sweeps_lambda : a.n_sw;
        void *args[] = {(void *)&a};
        HIP_TRY(hipLaunchKernel(h->roll.fn, dim3(count), dim3(nmpc::kWave * h->roll.waves), args,
                                h->roll.lds, h->stream));
    }
    if (check) {
        // fork (queued after the rollout, so the rollout's workgroups are
        // placed first): the cold start into buffer 1 (iteration state
        // untouched) and its residual into slot 1 on the side stream, while
        // the main stream builds and evaluates the supplied start
        HIP_TRY(hipStreamWaitEvent(h->side, h->ev_fork, 0));
        InitArgs ic = ia;
        ic.wx = ic.wu = ic.wl = nullptr;
        ic.X = h->X(1); ic.U = h->U(1); ic.LAM = h->L(1);
        ic.trajectory_only = 1;
        ic.pad_only = 0;
        // with one reference for all stages only stage 0 is evaluated, which
        // reads stages 0 and 1 (the instances that fall back get the cold start
        // written into buffer 0 by the choice)
        ic.nst = !h->opt.xref_per_stage && h->N > 2 ? 2 : 0;
        void *args[] = {(void *)&ic};
        HIP_TRY(hipLaunchKernel(nmpc::init_kernel(),
                                dim3(launch_grid((size_t)count * (ic.nst ? ic.nst : h->N) * h->np)),
                                dim3(256), args, 0, h->side));
        // with one reference for all stages the cold start's stage residuals
        // are all equal (x_i = x0, u = 0, lambda = 0): stage 0 stands for all
        const int rc = launch_residual(h, count, 1, 1, h->side, !h->opt.xref_per_stage);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(h->ev_join, h->side));
    }
    h->last_start_kind = kind;
    h->last_fallback = false;
    if (check) {
        // an input-built start has its residual from the rollout pass
        if (kind != kStartInputs) {
            int rc = launch_residual(h, count, 0, 0);
            if (rc) return rc;
        }
        HIP_TRY(hipStreamWaitEvent(h->stream, h->ev_join, 0));   // join
        IterArgs a = iter_args(h, count);
        a.units = count;
        a.res_first_stage = !h->opt.xref_per_stage;
        int *st = h->d_start;
        int used = kind;
        {
            void *args[] = {(void *)&a, (void *)&st, (void *)&used};
            HIP_TRY(hipLaunchKernel(nmpc::choose_flags_kernel(), dim3((count + 255) / 256),
                                    dim3(256), args, 0, h->stream));
        }
        {
            void *args[] = {(void *)&a, (void *)&st};
            HIP_TRY(hipLaunchKernel(nmpc::choose_copy_kernel(), dim3((unsigned)(count * h->N)),
                                    dim3(256), args, 0, h->stream));
        }
        h->last_fallback = true;
    }
    return NMPC_OK;
}

// Run the upper iteration for `count` instances whose x0/xref already sit in
// the handle's buffers; S^0 from the warm pointers (device, dense) or cold.
// Streaming scratch layout in d_stream (doubles): 10 per-point arrays
// [B][N][n], sc [B][N][ly][nsx], kun and v3 [B][N][m], row maxima (two
// 64-bit words per row) and row partials [B][N][nsy][kMaxLx].
size_t stream_doubles(const nmpc_handle *h)
{
    const size_t B = h->max_batch, N = h->N, n = h->n, m = h->m;
    const size_t lunits = (size_t)((h->prob.nsx + nmpc::kLowerCols - 1) / nmpc::kLowerCols) *
                          ((h->prob.nsy + nmpc::kLowerRows - 1) / nmpc::kLowerRows);
    return 10 * B * N * n + B * N * h->prob.ly * h->prob.nsx + 2 * B * N * m +
           B * N * h->prob.nsy * nmpc::kMaxLx + B * N * lunits * (2 * nmpc::kMaxM + 2);
}

nmpc::StreamArgs stream_args(const nmpc_handle *h, int count)
{
    nmpc::StreamArgs a{};
    const nmpc_problem &p = h->prob;
    a.P.nsx = p.nsx; a.P.nsy = p.nsy; a.P.n = h->n; a.P.N = h->N; a.P.m = h->m;
    a.P.lx = p.lx; a.P.ly = p.ly;
    a.P.h = p.h; a.P.k0 = p.k0; a.P.k1 = p.k1; a.P.q = p.q; a.P.r = p.r; a.P.gamma = p.gamma;
    a.P.tau = p.tau; a.P.ulo = p.u_lo; a.P.uhi = p.u_hi;
    a.apart = h->d_apart;
    const double dx = 1.0 / (p.nsx + 1), dy = 1.0 / (p.nsy + 1);
    a.P.idx2 = 1.0 / (dx * dx);
    a.P.idy2 = p.dim == 2 ? 1.0 / (dy * dy) : 0.0;
    a.P.c0 = 2.0 * a.P.idx2 + 2.0 * a.P.idy2;
    a.gx = h->d_gx; a.gy = h->d_gy;
    a.x0 = h->d_x0; a.xref = h->d_xref;
    a.xref_inst_stride = (long long)h->xref_len;
    a.xref_stage_stride = h->opt.xref_per_stage ? h->n : 0;
    for (int b = 0; b < 2; ++b) { a.X[b] = h->X(b); a.U[b] = h->U(b); a.LAM[b] = h->L(b); }
    const size_t B = h->max_batch, N = h->N, n = h->n, m = h->m;
    double *q = h->d_stream;
    double **arr[10] = {&a.b1, &a.b2, &a.invd, &a.cpk, &a.g2, &a.y5, &a.ytmp, &a.y4, &a.y4tmp, &a.cp};
    for (double **x : arr) { *x = q; q += B * N * n; }
    a.sc = q; q += B * N * p.ly * p.nsx;
    a.kun = q; q += B * N * m;
    a.v3 = q; q += B * N * m;
    a.rowt = q; q += B * N * p.nsy * nmpc::kMaxLx;
    a.nstrip = (p.nsx + nmpc::kLowerCols - 1) / nmpc::kLowerCols;
    a.nrb = (p.nsy + nmpc::kLowerRows - 1) / nmpc::kLowerRows;
    a.part = q; q += B * N * a.nrb * a.nstrip * nmpc::kMaxM;
    a.part2 = q; q += B * N * a.nrb * a.nstrip * nmpc::kMaxM;
    a.unorm = reinterpret_cast<unsigned long long *>(q);
    a.lunits = (long long)count * h->N * a.nrb * a.nstrip;
    a.lper_xcd = (int)(((a.lunits + 3) / 4 + 7) / 8);
    a.rst = h->d_rst;
    a.pst = h->d_rst + B * N;
    a.st = h->d_st; a.work = h->d_work; a.iters = h->d_iters; a.rfin = h->d_rfin; a.ctr = h->d_ctr;
    a.du = h->d_du;
    a.res_paper = h->opt.residual == NMPC_RES_PAPER;
    a.count = count;
    a.units = (long long)count * h->N * ((p.nsy + nmpc::kStreamRows - 1) / nmpc::kStreamRows);
    a.per_xcd = (int)((a.units + 7) / 8);
    a.tol = h->opt.tol; a.max_iter = h->opt.max_iter;
    a.n_sw = h->opt.n_sweep; a.n_schur = h->opt.n_schur;
    return a;
}

// One streaming upper iteration of precision `prec` (10 launches with the
// default schedule: two sweeps per solve take the fused lower-layer pass),
// queued on s.
int launch_stream_iteration(nmpc_handle *h, int prec, const nmpc::StreamArgs &a, hipStream_t s)
{
    const nmpc::StreamKernels k = nmpc::stream_kernels(prec);
    const dim3 rows(8 * a.per_xcd), stages(a.count * h->N), inst((a.count + 255) / 256);
    // LDS of the row-block passes: the residual pass stages two FP64 arrays,
    // the sweep passes two (one for F_x^T) arrays of T
    const int tsz = prec == nmpc::kModeFp32 ? 4 : 8;
    const size_t lds = nmpc::stream_lds_bytes(h->prob.nsx, tsz, 2);
    const dim3 lower(8 * a.lper_xcd);   // strip units (residual and fused lower passes)
    const size_t lds_jft = nmpc::stream_lds_bytes(h->prob.nsx, tsz, 1);
    auto go = [&](const void *fn, dim3 grid, int block, void **args, size_t sh = 0) -> int {
        HIP_TRY(hipLaunchKernel(fn, grid, dim3(block), args, sh, s));
        return NMPC_OK;
    };
    int rc;
    if (h->opt.n_sweep == 2) {
        // fused lower layer: one pass per Schur step and one for the final
        // block; the first Schur step (v3 = 0) rides in the residual pass
        const bool first_in_res = h->opt.n_schur >= 1;
        {
            void *args[] = {(void *)&a};
            if ((rc = go(first_in_res ? k.res1 : k.res, lower, 256, args))) return rc;
            if ((rc = go(k.stage, stages, 256, args))) return rc;
            if ((rc = go(k.decide, dim3(a.count), nmpc::kWave, args))) return rc;
        }
        // each lower pass forms v3 from the previous step's partials: those of
        // the residual pass's step are in part2, and the steps alternate
        for (int sch = first_in_res ? 1 : 0; sch <= h->opt.n_schur; ++sch) {
            const bool fin = sch == h->opt.n_schur;
            int which = sch == 0 ? -1 : (sch & 1);
            void *args[] = {(void *)&a, (void *)&which};
            if ((rc = go(fin ? k.lower_fin : k.lower, lower, 256, args))) return rc;
        }
        void *args[] = {(void *)&a};
        if (h->prob.tau > 0.0) {   // input box: cut the step by the rule
            if ((rc = go(k.box_lim, stages, nmpc::kWave, args))) return rc;
            if ((rc = go(k.box_apply, stages, 256, args))) return rc;
        }
        return go(k.advance, inst, 256, args);
    }
    const int passes = 1 + std::max(0, h->opt.n_sweep - 2);
    const int y5_tmp = (passes - 1) & 1;
    {
        void *args[] = {(void *)&a};
        if ((rc = go(k.res, lower, 256, args))) return rc;
        if ((rc = go(k.stage, stages, 256, args))) return rc;
        if ((rc = go(k.decide, dim3(a.count), nmpc::kWave, args))) return rc;
    }
    for (int sch = 0; sch <= h->opt.n_schur; ++sch) {
        const bool fin = sch == h->opt.n_schur;   // the final block after the Schur loop
        int use_v3 = (sch > 0 || fin) ? 1 : 0;
        if (use_v3) {
            int which = 1;
            void *args[] = {(void *)&a, (void *)&which};
            if ((rc = go(k.bsep, stages, 256, args))) return rc;
        }
        int sgn = fin ? 1 : -1;
        for (int pass = 0; pass < passes; ++pass) {
            void *args[] = {(void *)&a, (void *)&sgn, (void *)&use_v3, (void *)&pass};
            if ((rc = go(k.jf, rows, 256, args, lds))) return rc;
        }
        int ytmp = y5_tmp;
        {
            void *args[] = {(void *)&a, (void *)&sgn, (void *)&ytmp};
            if ((rc = go(k.axx, rows, 256, args, lds))) return rc;
        }
        for (int pass = 0; pass < passes; ++pass) {
            int last = pass == passes - 1, partials = fin ? 0 : 1, update = fin ? 1 : 0;
            void *args[] = {(void *)&a, (void *)&pass, (void *)&last, (void *)&partials,
                            (void *)&update, (void *)&ytmp};
            if ((rc = go(k.jft, rows, 256, args, lds_jft))) return rc;
        }
        if (!fin) {
            void *args[] = {(void *)&a};
            if ((rc = go(k.v3, stages, 256, args))) return rc;
        }
    }
    void *args[] = {(void *)&a};
    if (h->prob.tau > 0.0) {   // input box: cut the step by the rule
        if ((rc = go(k.box_lim, stages, nmpc::kWave, args))) return rc;
        if ((rc = go(k.box_apply, stages, 256, args))) return rc;
    }
    return go(k.advance, inst, 256, args);
}

int ensure_stream_graph(nmpc_handle *h, int prec, int count)
{
    const int len = h->opt.check_every;
    if (h->gexec[prec] && h->graph_count[prec] == count && h->graph_len[prec] == len)
        return NMPC_OK;
    if (h->gexec[prec]) { (void)hipGraphExecDestroy(h->gexec[prec]); h->gexec[prec] = nullptr; }
    if (h->graph[prec]) { (void)hipGraphDestroy(h->graph[prec]); h->graph[prec] = nullptr; }
    const nmpc::StreamArgs a = stream_args(h, count);
    HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    int rc = NMPC_OK;
    for (int t = 0; t < len && rc == NMPC_OK; ++t) rc = launch_stream_iteration(h, prec, a, h->stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->stream, &g);
    if (rc != NMPC_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return fail(NMPC_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    h->graph[prec] = g;
    HIP_TRY(hipGraphInstantiate(&h->gexec[prec], g, nullptr, nullptr, 0));
    h->graph_count[prec] = count; h->graph_len[prec] = len;
    return NMPC_OK;
}

// Each instance's returned iterate (buffer iters[b] & 1) to the outputs.
int launch_output(nmpc_handle *h, int count, double *ox, double *ou, double *ol)
{
    OutArgs oa{};
    oa.count = count; oa.N = h->N; oa.m = h->m; oa.iters = h->d_iters;
    oa.nsx = h->prob.nsx; oa.nsy = h->prob.nsy; oa.sx = h->sx;
    for (int b = 0; b < 2; ++b) { oa.X[b] = h->X(b); oa.U[b] = h->U(b); oa.LAM[b] = h->L(b); }
    oa.ox = ox; oa.ou = ou; oa.ol = ol;
    oa.vec = h->prob.nsx % 2 == 0 && h->sx % 2 == 0 &&
             ((uintptr_t)ox % 16) == 0 && ((uintptr_t)ol % 16) == 0;
    void *args[] = {(void *)&oa};
    const int per = oa.vec ? h->n / 2 : h->n;   // threads' items per unit
    const unsigned gx = (unsigned)std::min(64, (per + 255) / 256);
    const unsigned gy = (unsigned)std::min(count * h->N, 65535);
    HIP_TRY(hipLaunchKernel(nmpc::output_kernel(), dim3(gx, gy), dim3(256), args, 0, h->stream));
    return NMPC_OK;
}

// Gauss-Seidel upper layer: one launch per precision phase, one workgroup
// per instance; the kernels take every decision themselves.
int run_gs(nmpc_handle *h, int count)
{
    IterArgs a = iter_args(h, count);
    a.units = count;
    int upper = h->opt.upper;
    void *args[] = {(void *)&a, (void *)&upper};
    if (h->timing) HIP_TRY(hipEventRecord(h->t0, h->stream));
    int launches = 0;
    for (int prec : {nmpc::kModeFp32, nmpc::kModeFp64}) {
        if (prec == nmpc::kModeFp32 && main_prec(h->opt) != nmpc::kModeFp32) continue;
        // every instance leaves the FP32 kernel finished when it returns S^j
        if (prec == nmpc::kModeFp64 && main_prec(h->opt) == nmpc::kModeFp32 && h->opt.fp32_finish)
            continue;
        const nmpc_handle::Kern &k = h->gs[prec];
        a.gs_pf = k.pf;
        HIP_TRY(hipLaunchKernel(k.fn, dim3(count), dim3(nmpc::kWave * k.waves), args, k.lds,
                                h->stream));
        ++launches;
    }
    if (h->timing) {
        HIP_TRY(hipEventRecord(h->t1, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, h->t0, h->t1));
        h->kernel_ms += ms;
        h->launches += launches;
    }
    return NMPC_OK;
}

int run(nmpc_handle *h, int count, const double *wx, const double *wu, const double *wl,
        double *ox, double *ou, double *ol)
{
    {
        const int rc = build_start(h, count, wx, wu, wl);
        if (rc) return rc;
    }
    if (h->opt.upper != NMPC_UPPER_JACOBI) {
        const int rc = run_gs(h, count);
        if (rc) return rc;
        return launch_output(h, count, ox, ou, ol);
    }
    // Phase FP32 (FP32-sweep precision) runs until no instance is left in
    // FP32 mode, then phase FP64 until every instance has finished. Each
    // phase ends by max_iter + 4 launches; launches after an instance has
    // finished (or while it waits for the other phase) are no-ops for it.
    int prec = h->opt.precision == NMPC_FP32_SWEEP ? nmpc::kModeFp32 : nmpc::kModeFp64;
    const long long cap = 2 * ((long long)h->opt.max_iter + 8 + h->opt.check_every);
    long long launched = 0;
    // the first graph sized from the previous solve when its FP32 launches
    // and the FP64 phase fit in one graph of check_every launches
    bool first = prec == nmpc::kModeFp32 && !h->streaming && !h->opt.fp32_finish &&
                 h->last_iters >= 0 && h->last_iters + 4 <= h->opt.check_every;
    for (;;) {
        const int q = first ? 2 : prec;
        int rc = first ? ensure_first_graph(h, count, h->last_iters + 1)
                       : h->streaming ? ensure_stream_graph(h, prec, count) : ensure_graph(h, prec, count);
        if (rc != NMPC_OK) return rc;
        first = false;
        if (h->timing) HIP_TRY(hipEventRecord(h->t0, h->stream));
        HIP_TRY(hipGraphLaunch(h->gexec[q], h->stream));
        if (h->timing) HIP_TRY(hipEventRecord(h->t1, h->stream));
        launched += h->graph_len[q];
        HIP_TRY(hipMemcpyAsync(h->h_poll, h->d_ctr + 2, 2 * sizeof(int), hipMemcpyDeviceToHost,
                               h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        if (h->timing) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, h->t0, h->t1));
            h->kernel_ms += ms;
            h->launches += h->graph_len[q];
        }
        if (h->h_poll[0] >= count) break;
        if (prec == nmpc::kModeFp32 && h->h_poll[1] <= 0) prec = nmpc::kModeFp64;
        if (launched > cap)
            return fail(NMPC_E_DEVICE, "instances did not finish within max_iter launches");
    }
    return launch_output(h, count, ox, ou, ol);
}

}  // namespace

namespace nmpc {

// err_vs_fp64 of one result: 0 for FP64 solves; for FP32-sweep solves the
// size of the FP64 correction step taken from the iterate accepted in the FP32
// phase, max |du| / max |u^{j+1}| over the horizon; -1 where no such step was
// taken (fp32_finish, or the solve ended in the FP32 phase).
double fp32_step_error(bool fp32, bool finish, const InstState &s, const unsigned long long *du)
{
    if (!fp32) return 0.0;
    if (finish || s.mode != nmpc::kModeFp64) return -1.0;
    double d, u;
    std::memcpy(&d, &du[0], sizeof d);
    std::memcpy(&u, &du[1], sizeof u);
    return u > 0.0 ? d / u : d;
}

// Evaluation-only visits of one finished instance (R14): the check of the
// FP64-corrected iterate in an FP32-sweep solve, one per instance that
// reached it (final mode FP64 with no correction still owed). The streaming
// path counts updates only and reports none.
int eval_only_visits(bool fp32, bool finish, bool streaming, const InstState &s)
{
    return fp32 && !finish && !streaming && s.mode == nmpc::kModeFp64 && !s.pending ? 1 : 0;
}

}  // namespace nmpc

namespace {

int collect_info(nmpc_handle *h, int count, nmpc_info *info)
{
    // the final state lives in the parity slot of the last kernel + 1; the
    // status is sticky once set, so both slots come back and the final one
    // is taken. Everything of the batch is gathered on the device first and
    // read with one copy into pinned memory.
    nmpc::PackArgs pa{h->d_st, h->d_iters, h->d_rfin, h->d_du,
                      h->last_fallback ? h->d_start : nullptr, count, h->max_batch, h->d_info};
    void *pargs[] = {(void *)&pa};
    HIP_TRY(hipLaunchKernel(nmpc::info_pack_kernel(), dim3((count + 255) / 256), dim3(256), pargs, 0,
                            h->stream));
    HIP_TRY(hipMemcpyAsync(h->h_info, h->d_info, sizeof(nmpc::InfoPack) * count,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    int worst = NMPC_OK, most = 0;
    for (int b = 0; b < count; ++b) {
        const nmpc::InfoPack &pk = h->h_info[b];
        const InstState &s = pk.s[0].status != nmpc::kActive ? pk.s[0] : pk.s[1];
        most = std::max(most, pk.iters);
        if (h->timing) {
            const int eo = nmpc::eval_only_visits(h->opt.precision == NMPC_FP32_SWEEP,
                                                  h->opt.fp32_finish != 0, h->streaming, s);
            h->units += (long long)(s.e - eo) * h->N;
            h->units_eval += (long long)eo * h->N;
        }
        const int status = s.status == nmpc::kActive ? NMPC_E_DEVICE : s.status;
        if (info) {
            info[b].r_scaled = pk.rf[0];
            info[b].r_paper = pk.rf[1];
            info[b].iters = pk.iters;
            info[b].status = status;
            info[b].fp32_iters = s.f32;
            info[b].start_used = h->last_fallback ? pk.used : h->last_start_kind;
            info[b].err_vs_fp64 = nmpc::fp32_step_error(main_prec(h->opt) == nmpc::kModeFp32,
                                                  h->opt.fp32_finish != 0, s, pk.du);
        }
        if (status != NMPC_OK && worst == NMPC_OK) worst = status;
    }
    h->last_iters = worst == NMPC_OK ? most : -1;
    return worst;
}

}  // namespace

extern "C" {

void nmpc_default_options(nmpc_options *opt)
{
    if (!opt) return;
    opt->tol = 1e-6;
    opt->max_iter = 2000;
    opt->n_sweep = 2;
    opt->n_schur = 2;
    opt->precision = NMPC_FP64;
    opt->check_every = 16;
    opt->xref_per_stage = 0;
    opt->tile_rows = 0;
    opt->warm_sweeps = 0;
    opt->fallback = 0;
    opt->upper = NMPC_UPPER_JACOBI;
    opt->path = NMPC_PATH_AUTO;
    opt->omega = 1.0;
    opt->fp32_finish = 0;
    opt->residual = NMPC_RES_SCALED;
    opt->warm_sweeps_lambda = 0;
}

}  // extern "C"

namespace {

// A dense-B problem: the heat model of the model engine, plus a staging area
// and a stream for host-buffer solves.
int create_dense(nmpc_handle *h, nmpc_handle **out)
{
    const nmpc_problem &p = h->prob;
    nmpc_model_problem mp{};
    mp.model = NMPC_MODEL_HEAT;
    mp.boundary = NMPC_BC_DIRICHLET;
    mp.nsx = p.nsx;
    mp.nsy = p.dim == 1 ? 1 : p.nsy;
    mp.horizon = p.horizon;
    mp.n_inputs = h->m;
    mp.B = p.B;
    mp.h = p.h; mp.q = p.q; mp.qv = 0.0; mp.r = p.r; mp.gamma = p.gamma;
    mp.tau = p.tau; mp.u_lo = p.u_lo; mp.u_hi = p.u_hi; mp.u_cold = 0.0;
    mp.k0 = p.k0; mp.k1 = p.k1; mp.damp = 0.0;
    int rc = nmpc_model_create(&mp, &h->opt, h->max_batch, &h->dense);
    if (rc) { delete h; return rc; }
    h->prob.B = nullptr;
    h->prob.gx = h->prob.gy = nullptr;
    hipError_t e = hipMalloc((void **)&h->d_out,
                             sizeof(double) * ((size_t)h->N * (2 * (size_t)h->n + h->m) + 2 * h->n));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        release(h);
        return fail(e == hipErrorOutOfMemory ? NMPC_E_OOM : NMPC_E_DEVICE,
                    std::string("create: ") + hipGetErrorString(e));
    }
    *out = h;
    return NMPC_OK;
}

}  // namespace

extern "C" {

int nmpc_create(const nmpc_problem *prob, const nmpc_options *opt, int32_t max_batch,
                nmpc_handle **out)
{
    g_err.clear();
    if (!out) return fail(NMPC_E_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_problem(prob);
    if (rc) return rc;
    rc = check_options(opt);
    if (rc) return rc;
    if (max_batch < 1) return fail(NMPC_E_ARG, "max_batch must be >= 1");
    nmpc_handle *h = new (std::nothrow) nmpc_handle();
    if (!h) return fail(NMPC_E_OOM, "host allocation failed");
    h->prob = *prob;
    h->opt = *opt;
    h->max_batch = max_batch;
    h->n = prob->nsx * prob->nsy;
    h->m = prob->lx * prob->ly;
    h->N = prob->horizon;
    if (prob->b_kind == NMPC_B_DENSE) return create_dense(h, out);
    rc = choose_path(prob, opt, &h->streaming);
    if (rc) { delete h; return rc; }
    if (!h->streaming) {
        rc = select_all(prob, opt, h->kern, h->gs);
        if (rc) { delete h; return rc; }
    }
    h->gx.assign(prob->gx, prob->gx + (size_t)prob->lx * prob->nsx);
    h->gy.assign(prob->gy, prob->gy + (size_t)prob->ly * prob->nsy);
    h->prob.gx = h->gx.data();
    h->prob.gy = h->gy.data();
    if (!h->streaming) {
        TileCfg cfg{};
        h->roll.fn = nmpc::rollout_kernel(tile_cx(prob->nsx), prob->lx, prob->ly, &cfg);
        if (!h->roll.fn) { delete h; return fail(NMPC_E_UNSUPPORTED, "no rollout kernel instance"); }
        h->roll.cfg = cfg;
        h->roll.waves = (((prob->nsy + cfg.rows - 1) / cfg.rows) + 3) / 4;
        if (h->roll.waves > cfg.max_waves) { delete h; return fail(NMPC_E_UNSUPPORTED, "grid too tall"); }
        h->roll.lds = nmpc::lds_layout(h->roll.waves * 4, h->roll.waves, cfg.cx, 8, prob->lx,
                                       prob->ly, cfg.rows).total;
    }
    h->sx = h->streaming ? prob->nsx : 16 * h->kern[nmpc::kModeFp64].cfg.cx;
    h->np = h->sx * prob->nsy;
    h->xref_len = (size_t)h->np * (opt->xref_per_stage ? h->N : 1);
    const size_t B = max_batch, S = B * h->N * (2 * (size_t)h->np + h->m);
#define ALLOC(ptr, bytes)                                                          \
    do {                                                                           \
        hipError_t e_ = hipMalloc((void **)&(ptr), (bytes));                       \
        if (e_ != hipSuccess) {                                                    \
            release(h);                                                            \
            return fail(e_ == hipErrorOutOfMemory ? NMPC_E_OOM : NMPC_E_DEVICE,    \
                        std::string("hipMalloc: ") + hipGetErrorString(e_));       \
        }                                                                          \
    } while (0)
    ALLOC(h->d_gx, sizeof(double) * h->gx.size());
    ALLOC(h->d_gy, sizeof(double) * h->gy.size());
    ALLOC(h->d_S[0], sizeof(double) * S);
    ALLOC(h->d_S[1], sizeof(double) * S);
    ALLOC(h->d_x0, sizeof(double) * B * h->np);
    ALLOC(h->d_xref, sizeof(double) * B * (size_t)h->np * h->N);   // room for per-stage xref
    // dense staging of one instance (host-buffer solves): outputs, or x0 + xref
    ALLOC(h->d_out, sizeof(double) * (size_t)h->N * (2 * (size_t)h->n + h->m));
    ALLOC(h->d_rst, sizeof(unsigned long long) * 6 * B * h->N);
    ALLOC(h->d_st, sizeof(InstState) * 2 * B);
    ALLOC(h->d_iters, sizeof(int) * B);
    ALLOC(h->d_rfin, sizeof(double) * 2 * B);
    ALLOC(h->d_du, sizeof(unsigned long long) * 2 * B);
    ALLOC(h->d_ctr, sizeof(int) * 4);
    ALLOC(h->d_start, sizeof(int) * B);
    ALLOC(h->d_info, sizeof(nmpc::InfoPack) * B);
    if (prob->tau > 0.0) {
        ALLOC(h->d_apart, sizeof(double) * B * h->N);
        ALLOC(h->d_aupd, sizeof(int) * B);
    }
    if (h->streaming) {
        ALLOC(h->d_stream, sizeof(double) * stream_doubles(h));
        ALLOC(h->d_work, sizeof(int) * B);
        const size_t lds = nmpc::stream_lds_bytes(prob->nsx);
        for (int prec : {nmpc::kModeFp64, nmpc::kModeFp32}) {
            const nmpc::StreamKernels k = nmpc::stream_kernels(prec);
            for (const void *fn : {k.jf, k.axx, k.jft})
                if (lds > 48 * 1024 &&
                    hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
                    release(h);
                    return fail(NMPC_E_DEVICE, "streaming kernels: LDS limit");
                }
        }
    }

#undef ALLOC
    hipError_t e = hipHostMalloc((void **)&h->h_poll, 2 * sizeof(int), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&h->h_info, sizeof(nmpc::InfoPack) * B, hipHostMallocDefault);
    for (int prec : {nmpc::kModeFp64, nmpc::kModeFp32})
        for (const nmpc_handle::Kern *k : {&h->kern[prec], &h->gs[prec]})
            if (e == hipSuccess && k->fn && k->lds > 48 * 1024)
                e = hipFuncSetAttribute(k->fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)k->lds);
    if (e == hipSuccess && h->roll.fn && h->roll.lds > 48 * 1024)
        e = hipFuncSetAttribute(h->roll.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)h->roll.lds);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&h->t0);
    if (e == hipSuccess) e = hipEventCreate(&h->t1);

    if (e == hipSuccess)
        e = hipMemcpy(h->d_gx, h->gx.data(), sizeof(double) * h->gx.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(h->d_gy, h->gy.data(), sizeof(double) * h->gy.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(h->d_ctr, 0, sizeof(int) * 4);

    if (e != hipSuccess) {
        release(h);
        return fail(NMPC_E_DEVICE, std::string("create: ") + hipGetErrorString(e));
    }
    *out = h;
    return NMPC_OK;
}

int nmpc_set_options(nmpc_handle *h, const nmpc_options *opt)
{
    g_err.clear();
    if (!h) return fail(NMPC_E_ARG, "handle is NULL");
    int rc = check_options(opt);
    if (rc) return rc;
    if (h->dense) {
        rc = nmpc_model_set_options(h->dense, opt);
        if (rc == NMPC_OK) h->opt = *opt;
        return rc;
    }
    bool streaming = false;
    rc = choose_path(&h->prob, opt, &streaming);
    if (rc) return rc;
    if (streaming != h->streaming)
        return fail(NMPC_E_UNSUPPORTED, "set_options cannot switch between fused and streaming paths");
    nmpc_handle::Kern kn[2] = {}, gn[2] = {};
    if (!streaming) {
        rc = select_all(&h->prob, opt, kn, gn);
        if (rc) return rc;
    }
    for (int prec : {nmpc::kModeFp64, nmpc::kModeFp32}) {
        if ((rc = raise_lds(kn[prec]))) return rc;
        if ((rc = raise_lds(gn[prec]))) return rc;
    }
    h->kern[0] = kn[0];
    h->kern[1] = kn[1];
    h->gs[0] = gn[0];
    h->gs[1] = gn[1];
    if (opt->xref_per_stage != h->opt.xref_per_stage)
        h->xref_len = (size_t)h->np * (opt->xref_per_stage ? h->N : 1);
    h->opt = *opt;
    h->graph_count[0] = h->graph_count[1] = h->graph_count[2] = -1;   // recapture: options are kernel arguments
    h->last_iters = -1;
    return NMPC_OK;
}

int nmpc_solve(nmpc_handle *h, const double *x0, const double *xref, const double *warm_x,
               const double *warm_u, const double *warm_lam, double *out_x, double *out_u,
               double *out_lam, nmpc_info *info)
{
    g_err.clear();
    if (!h || !x0 || !xref || !out_x || !out_u || !out_lam)
        return fail(NMPC_E_ARG, "NULL argument");
    if (start_kind(warm_x, warm_u, warm_lam) < 0)
        return fail(NMPC_E_ARG, "warm start needs (x, u, lambda), u alone, or (u, lambda)");
    const size_t n = h->n, m = h->m, N = h->N;
    if (h->dense) {   // model engine: stage x0, xref, the start and the outputs in d_out
        double *dx0 = h->d_out + N * (2 * n + m), *dxr = dx0 + n;
        double *ox = h->d_out, *ol = h->d_out + N * n, *ou = h->d_out + 2 * N * n;
        HIP_TRY(hipMemcpyAsync(dx0, x0, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipMemcpyAsync(dxr, xref, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
        if (warm_x) {
            if (!warm_u || !warm_lam)
                return fail(NMPC_E_UNSUPPORTED, "dense-B problems take cold or (x, u, lambda) starts");
            HIP_TRY(hipMemcpyAsync(ox, warm_x, sizeof(double) * N * n, hipMemcpyHostToDevice, h->stream));
            HIP_TRY(hipMemcpyAsync(ol, warm_lam, sizeof(double) * N * n, hipMemcpyHostToDevice, h->stream));
            HIP_TRY(hipMemcpyAsync(ou, warm_u, sizeof(double) * N * m, hipMemcpyHostToDevice, h->stream));
        } else if (warm_u) {
            return fail(NMPC_E_UNSUPPORTED, "dense-B problems take cold or (x, u, lambda) starts");
        }
        nmpc_info tmp;
        // the model engine reads the start into its own buffers before writing the outputs
        const int rc = nmpc_model_solve_batch(h->dense, 1, dx0, dxr, warm_x ? ox : nullptr,
                                              warm_x ? ou : nullptr, warm_x ? ol : nullptr, ox,
                                              ou, ol, info ? info : &tmp, h->stream);
        if (rc != NMPC_OK && rc != NMPC_E_NOCONV && rc != NMPC_E_NONFINITE) return rc;
        HIP_TRY(hipMemcpyAsync(out_x, ox, sizeof(double) * N * n, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(out_lam, ol, sizeof(double) * N * n, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(out_u, ou, sizeof(double) * N * m, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        return rc;
    }
    // dense x0 | xref staged in d_out, then padded into the input buffers
    HIP_TRY(hipMemcpyAsync(h->d_out, x0, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->d_out + n, xref, sizeof(double) * h->xref_dense(),
                           hipMemcpyHostToDevice, h->stream));
    {
        const int rc = stage_inputs(h, 1, h->d_out, h->d_out + n);
        if (rc) return rc;
    }
    const double *wx = nullptr, *wu = nullptr, *wl = nullptr;
    // stage the dense start in the output staging area (read by k_init
    // before anything writes d_out again)
    double *stg = h->d_out;
    if (warm_x) {
        HIP_TRY(hipMemcpyAsync(stg, warm_x, sizeof(double) * N * n, hipMemcpyHostToDevice, h->stream));
        wx = stg;
    }
    if (warm_lam) {
        HIP_TRY(hipMemcpyAsync(stg + N * n, warm_lam, sizeof(double) * N * n, hipMemcpyHostToDevice, h->stream));
        wl = stg + N * n;
    }
    if (warm_u) {
        HIP_TRY(hipMemcpyAsync(stg + 2 * N * n, warm_u, sizeof(double) * N * m, hipMemcpyHostToDevice, h->stream));
        wu = stg + 2 * N * n;
    }
    double *ox = h->d_out, *ol = h->d_out + N * n, *ou = h->d_out + 2 * N * n;
    int rc = run(h, 1, wx, wu, wl, ox, ou, ol);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(out_x, ox, sizeof(double) * N * n, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(out_lam, ol, sizeof(double) * N * n, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(out_u, ou, sizeof(double) * N * m, hipMemcpyDeviceToHost, h->stream));
    nmpc_info tmp;
    return collect_info(h, 1, info ? info : &tmp);
}

int nmpc_solve_batch(nmpc_handle *h, int32_t count, const double *x0, const double *xref,
                     const double *warm_x, const double *warm_u, const double *warm_lam,
                     double *out_x, double *out_u, double *out_lam, nmpc_info *info,
                     void *stream)
{
    g_err.clear();
    if (!h || !x0 || !xref || !out_x || !out_u || !out_lam)
        return fail(NMPC_E_ARG, "NULL argument");
    if (count < 1 || count > h->max_batch) return fail(NMPC_E_ARG, "count outside 1..max_batch");
    if (start_kind(warm_x, warm_u, warm_lam) < 0)
        return fail(NMPC_E_ARG, "warm start needs (x, u, lambda), u alone, or (u, lambda)");
    if (h->dense)
        return nmpc_model_solve_batch(h->dense, count, x0, xref, warm_x, warm_u, warm_lam, out_x,
                                      out_u, out_lam, info, stream);
    hipStream_t us = (hipStream_t)stream;
    HIP_TRY(hipEventRecord(h->ev, us));
    HIP_TRY(hipStreamWaitEvent(h->stream, h->ev, 0));
    int rc = stage_inputs(h, count, x0, xref);
    if (rc) return rc;
    rc = run(h, count, warm_x, warm_u, warm_lam, out_x, out_u, out_lam);
    if (rc) return rc;
    std::vector<nmpc_info> tmp;
    if (!info) { tmp.resize(count); info = tmp.data(); }
    return collect_info(h, count, info);
}

int nmpc_residual_batch(nmpc_handle *h, int32_t count, const double *x0, const double *xref,
                        const double *x, const double *u, const double *lam, double *r_scaled,
                        double *r_paper, void *stream)
{
    g_err.clear();
    if (!h || !x0 || !xref || !x || !u || !lam || !r_scaled || !r_paper)
        return fail(NMPC_E_ARG, "NULL argument");
    if (count < 1 || count > h->max_batch) return fail(NMPC_E_ARG, "count outside 1..max_batch");
    if (h->dense)
        return nmpc_model_residual_batch(h->dense, count, x0, xref, x, u, lam, r_scaled, r_paper,
                                         stream);
    hipStream_t us = (hipStream_t)stream;
    HIP_TRY(hipEventRecord(h->ev, us));
    HIP_TRY(hipStreamWaitEvent(h->stream, h->ev, 0));
    int rc = stage_inputs(h, count, x0, xref);
    if (rc) return rc;
    {   // trajectories into buffer 0 (padded), via the warm-start path of k_init
        InitArgs ia{};
        ia.count = count; ia.B = h->max_batch; ia.N = h->N; ia.m = h->m;
        ia.nsx = h->prob.nsx; ia.nsy = h->prob.nsy; ia.sx = h->sx; ia.mode = nmpc::kModeFp64;
        ia.x0 = h->d_x0; ia.wx = x; ia.wu = u; ia.wl = lam;
        ia.X = h->X(0); ia.U = h->U(0); ia.LAM = h->L(0);
        ia.st = h->d_st; ia.iters = h->d_iters; ia.ctr = h->d_ctr;
        void *args[] = {(void *)&ia};
        HIP_TRY(hipLaunchKernel(nmpc::init_kernel(), dim3(launch_grid((size_t)count * h->N * h->np)),
                                dim3(256), args, 0, h->stream));
    }
    const unsigned long long *rst = nullptr, *pst = nullptr;
    if (h->streaming) {   // residual passes of the streaming path (stage norms in rst / pst)
        const nmpc::StreamArgs a = stream_args(h, count);
        const nmpc::StreamKernels k = nmpc::stream_kernels(nmpc::kModeFp64);
        void *a2[] = {(void *)&a};
        HIP_TRY(hipLaunchKernel(k.res, dim3(8 * a.lper_xcd), dim3(256), a2, 0, h->stream));
        HIP_TRY(hipLaunchKernel(k.stage, dim3(count * h->N), dim3(256), a2, 0, h->stream));
        rst = a.rst;
        pst = a.pst;
    } else {
        IterArgs a = iter_args(h, count);
        a.residual_only = 1;
        rc = launch_iterate(h, nmpc::kModeFp64, a, h->stream);
        if (rc) return rc;
        rst = a.rst;
        pst = a.pst;
    }
    const size_t per = (size_t)count * h->N;   // slot 0 of both arrays
    std::vector<unsigned long long> bits(2 * per);
    HIP_TRY(hipMemcpyAsync(bits.data(), rst, sizeof(unsigned long long) * per,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(bits.data() + per, pst, sizeof(unsigned long long) * per,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int b = 0; b < count; ++b) {
        unsigned long long ms = 0, mp = 0;   // bit-pattern max: NaN above all finite values
        for (int i = 0; i < h->N; ++i) {
            ms = std::max(ms, bits[(size_t)b * h->N + i]);
            mp = std::max(mp, bits[per + (size_t)b * h->N + i]);
        }
        std::memcpy(&r_scaled[b], &ms, sizeof(double));
        std::memcpy(&r_paper[b], &mp, sizeof(double));
    }
    return NMPC_OK;
}

void nmpc_destroy(nmpc_handle *h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    release(h);
}

const char *nmpc_strerror(int code)
{
    switch (code) {
    case NMPC_OK: return "ok";
    case NMPC_E_ARG: return "invalid argument";
    case NMPC_E_NOCONV: return "not converged within max_iter";
    case NMPC_E_NONFINITE: return "residual became non-finite";
    case NMPC_E_DEVICE: return "HIP device error";
    case NMPC_E_OOM: return "out of device memory";
    case NMPC_E_UNSUPPORTED: return "unsupported problem shape";
    default: return "unknown error";
    }
}

const char *nmpc_last_error(void) { return g_err.c_str(); }

void nmpc_set_last_error(const char *msg) { g_err = msg ? msg : ""; }

int nmpc_timing_enable(nmpc_handle *h, int32_t enable)
{
    g_err.clear();
    if (!h) return fail(NMPC_E_ARG, "handle is NULL");
    if (h->dense) return nmpc_model_timing_enable(h->dense, enable);
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->timing = enable != 0;
    if (h->timing) {
        h->kernel_ms = 0.0;
        h->launches = 0;
        h->units = 0;
        h->units_eval = 0;
    }
    return NMPC_OK;
}

int nmpc_timing_read(const nmpc_handle *h, double *kernel_ms, int64_t *launches, int64_t *units)
{
    g_err.clear();
    if (!h) return fail(NMPC_E_ARG, "handle is NULL");
    if (h->dense) return nmpc_model_timing_read(h->dense, kernel_ms, launches, units);
    if (kernel_ms) *kernel_ms = h->kernel_ms;
    if (launches) *launches = h->launches;
    if (units) *units = (int64_t)h->units;
    return NMPC_OK;
}

int nmpc_timing_read_eval(const nmpc_handle *h, int64_t *eval_units)
{
    g_err.clear();
    if (!h) return fail(NMPC_E_ARG, "handle is NULL");
    if (eval_units) *eval_units = h->dense ? 0 : (int64_t)h->units_eval;
    return NMPC_OK;
}

int nmpc_autotune(nmpc_handle *h, int32_t count, const double *x0, const double *xref,
                  int32_t iters, void *stream, int32_t *tile_rows)
{
    g_err.clear();
    if (!h || !x0 || !xref) return fail(NMPC_E_ARG, "NULL argument");
    if (h->dense) return fail(NMPC_E_UNSUPPORTED, "dense-B problems have no tile to tune");
    if (count < 1 || count > h->max_batch) return fail(NMPC_E_ARG, "count outside 1..max_batch");
    if (iters < 1 || iters > 1000) return fail(NMPC_E_ARG, "iters must be 1..1000");
    if (h->streaming) return fail(NMPC_E_UNSUPPORTED, "the streaming path has no tile choices");
    const int prec = h->opt.precision == NMPC_FP32_SWEEP ? nmpc::kModeFp32 : nmpc::kModeFp64;
    hipStream_t us = (hipStream_t)stream;
    HIP_TRY(hipEventRecord(h->ev, us));
    HIP_TRY(hipStreamWaitEvent(h->stream, h->ev, 0));
    int rc = stage_inputs(h, count, x0, xref);
    if (rc) return rc;
    const bool gs = h->opt.upper != NMPC_UPPER_JACOBI;
    nmpc_handle::Kern &slot = gs ? h->gs[prec] : h->kern[prec];
    const nmpc_handle::Kern keep = slot;
    int best_ry = -1;
    float best_ms = 0.f;
    nmpc_handle::Kern best{};
    for (int ry = 1; ry <= 16; ++ry) {
        nmpc_handle::Kern k;
        if (select_kernel(&h->prob, prec, ry, &k, gs) != NMPC_OK) continue;   // no such tile
        if ((rc = raise_lds(k))) return rc;
        slot = k;
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {   // the first pass loads code and warms caches
            rc = build_start(h, count, nullptr, nullptr, nullptr);
            if (rc) { slot = keep; return rc; }
            IterArgs a = iter_args(h, count);
            HIP_TRY(hipEventRecord(h->t0, h->stream));
            if (gs) {   // `iters` iterations of the main-precision kernel, no early exit
                a.units = count;
                a.tol = -1.0;
                a.max_iter = iters;
                a.gs_pf = k.pf;
                int upper = h->opt.upper;
                void *args[] = {(void *)&a, (void *)&upper};
                HIP_TRY(hipLaunchKernel(k.fn, dim3(count), dim3(nmpc::kWave * k.waves), args,
                                        k.lds, h->stream));
            } else {
                for (int t = 0; t < iters && rc == NMPC_OK; ++t) {
                    a.kofs = t;
                    rc = launch_iterate(h, prec, a, h->stream);
                }
            }
            if (rc) { slot = keep; return rc; }
            HIP_TRY(hipEventRecord(h->t1, h->stream));
            HIP_TRY(hipStreamSynchronize(h->stream));
            HIP_TRY(hipEventElapsedTime(&ms, h->t0, h->t1));
        }
        if (best_ry < 0 || ms < best_ms) { best_ry = ry; best_ms = ms; best = k; }
    }
    g_err.clear();
    if (best_ry < 0) { slot = keep; return fail(NMPC_E_UNSUPPORTED, "no tile to tune"); }
    slot = best;
    h->opt.tile_rows = best_ry;
    h->graph_count[0] = h->graph_count[1] = h->graph_count[2] = -1;
    if (tile_rows) *tile_rows = best_ry;
    return NMPC_OK;
}

int nmpc_shift_batch(nmpc_handle *h, int32_t count, const double *x, const double *u,
                     const double *lam, double *out_x, double *out_u, double *out_lam,
                     void *stream)
{
    g_err.clear();
    if (!h || !x || !u || !lam || !out_x || !out_u || !out_lam) return fail(NMPC_E_ARG, "NULL argument");
    if (count < 1 || count > h->max_batch) return fail(NMPC_E_ARG, "count outside 1..max_batch");
    if (out_x == x || out_u == u || out_lam == lam)
        return fail(NMPC_E_ARG, "shift outputs must not alias the inputs");
    long long cnt = count;
    int N = h->N;
    const double *src[3] = {x, u, lam};
    double *dst[3] = {out_x, out_u, out_lam};
    const long long w[3] = {h->n, h->m, h->n};
    for (int q = 0; q < 3; ++q) {
        long long ww = w[q];
        void *args[] = {(void *)&src[q], (void *)&dst[q], (void *)&cnt, (void *)&N, (void *)&ww};
        HIP_TRY(hipLaunchKernel(nmpc::shift_kernel(), dim3(launch_grid((size_t)cnt * N * ww)),
                                dim3(256), args, 0, (hipStream_t)stream));
    }
    return NMPC_OK;
}

int nmpc_plant_step_batch(nmpc_handle *h, int32_t count, const double *x, const double *u,
                          int32_t ldu, double dt, double *out, void *stream)
{
    g_err.clear();
    if (!h || !x || !u || !out) return fail(NMPC_E_ARG, "NULL argument");
    if (h->dense) return fail(NMPC_E_UNSUPPORTED, "the plant step takes the Kronecker input form");
    if (count < 1 || count > h->max_batch) return fail(NMPC_E_ARG, "count outside 1..max_batch");
    if (ldu < h->m) return fail(NMPC_E_ARG, "ldu smaller than the number of inputs");
    if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(NMPC_E_ARG, "dt must be finite and >= 0");
    if (out == x) return fail(NMPC_E_ARG, "plant output must not alias x");
    nmpc::PlantArgs a{};
    const nmpc_problem &p = h->prob;
    a.count = count; a.nsx = p.nsx; a.nsy = p.nsy; a.lx = p.lx; a.ly = p.ly; a.ldu = ldu;
    a.x = x; a.u = u; a.gx = h->d_gx; a.gy = h->d_gy; a.out = out;
    a.dt = dt; a.k0 = p.k0; a.k1 = p.k1;
    const double dx = 1.0 / (p.nsx + 1), dy = 1.0 / (p.nsy + 1);
    a.idx2 = 1.0 / (dx * dx);
    a.idy2 = p.dim == 2 ? 1.0 / (dy * dy) : 0.0;
    void *args[] = {(void *)&a};
    HIP_TRY(hipLaunchKernel(nmpc::plant_kernel(), dim3(launch_grid((size_t)count * h->n)), dim3(256),
                            args, 0, (hipStream_t)stream));
    return NMPC_OK;
}

int nmpc_kernel_config(const nmpc_handle *h, int32_t *rows_per_lane, int32_t *waves,
                       int32_t *workgroups)
{
    if (!h) return NMPC_E_ARG;
    if (h->dense) {   // model engine: one workgroup per instance
        if (rows_per_lane) *rows_per_lane = 0;
        if (waves) *waves = 0;
        if (workgroups) *workgroups = h->max_batch;
        return NMPC_OK;
    }
    if (h->streaming) {   // one 256-thread workgroup per grid row of every stage
        if (rows_per_lane) *rows_per_lane = 0;
        if (waves) *waves = 4;
        if (workgroups) *workgroups = h->max_batch * h->N * h->prob.nsy;
        return NMPC_OK;
    }
    const int prec = main_prec(h->opt);
    const bool gs = h->opt.upper != NMPC_UPPER_JACOBI;
    const nmpc_handle::Kern &k = gs ? h->gs[prec] : h->kern[prec];
    if (rows_per_lane) *rows_per_lane = k.cfg.rows;
    if (waves) *waves = k.waves;
    if (workgroups) *workgroups = gs ? h->max_batch : 8 * ((h->max_batch * h->N + 7) / 8);
    return NMPC_OK;
}

}  // extern "C"
