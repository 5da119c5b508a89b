// nmpc_model_runtime.hip -- host side and C ABI of the model engine: problem
// checks, device workspace, launches on the caller's stream, results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "nmpc.h"
#include "nmpc_model.h"

struct nmpc_model {
    nmpc_model_problem prob{};
    nmpc_options opt{};
    int max_batch = 0;
    int nodes = 0, nxg = 0, m = 0, N = 0;
    int ppt = 1, threads = 64;
    size_t lds = 0;
    std::vector<int> act, nodeinp;
    int *d_nodeinp = nullptr, *d_act = nullptr;
    double *d_B = nullptr;
    double *d_X[2] = {nullptr, nullptr}, *d_U[2] = {nullptr, nullptr}, *d_L[2] = {nullptr, nullptr};
    double *d_lim = nullptr, *d_info_d = nullptr;
    int *d_info_i = nullptr;
    bool timing = false;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    double kernel_ms = 0.0;
    long long launches = 0, units = 0;
};

namespace {

int mfail(int code, const std::string &msg)
{
    nmpc_set_last_error(msg.c_str());
    return code;
}

#define MODEL_TRY(expr)                                                               \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return mfail(e_ == hipErrorOutOfMemory ? NMPC_E_OOM : NMPC_E_DEVICE,      \
                         std::string(#expr) + ": " + hipGetErrorString(e_));          \
    } while (0)

bool fin(double v) { return std::isfinite(v); }

int check_model(const nmpc_model_problem *p)
{
    if (!p) return mfail(NMPC_E_ARG, "model problem is NULL");
    if (p->model < NMPC_MODEL_HEAT || p->model > NMPC_MODEL_WAVE)
        return mfail(NMPC_E_ARG, "model must be NMPC_MODEL_HEAT, _PLATE or _WAVE");
    if (p->boundary != NMPC_BC_DIRICHLET && p->boundary != NMPC_BC_NEUMANN)
        return mfail(NMPC_E_ARG, "boundary must be NMPC_BC_DIRICHLET or NMPC_BC_NEUMANN");
    if (p->nsx < 1 || p->nsy < 1 || p->horizon < 1 || p->n_inputs < 1)
        return mfail(NMPC_E_ARG, "nsx, nsy, horizon and n_inputs must be >= 1");
    if (p->boundary == NMPC_BC_NEUMANN && (p->nsx < 2 || (p->nsy != 1 && p->nsy < 2)))
        return mfail(NMPC_E_ARG, "Neumann boundaries need at least 2 nodes per axis");
    if ((long long)p->nsx * p->nsy > nmpc::kModelMaxNodes)
        return mfail(NMPC_E_UNSUPPORTED, "the model engine takes up to 4096 grid nodes");
    if (p->n_inputs > nmpc::kModelMaxM || p->horizon > nmpc::kModelMaxN)
        return mfail(NMPC_E_UNSUPPORTED, "the model engine takes up to 64 inputs and 256 stages");
    if (!(fin(p->h) && p->h > 0.0 && fin(p->r) && p->r > 0.0 && fin(p->q) && p->q >= 0.0 &&
          fin(p->qv) && p->qv >= 0.0 && fin(p->gamma) && p->gamma >= 0.0))
        return mfail(NMPC_E_ARG, "h, r > 0 and q, qv, gamma >= 0 must be finite");
    if (!(fin(p->tau) && p->tau >= 0.0))
        return mfail(NMPC_E_ARG, "tau must be finite and >= 0");
    if (p->tau > 0.0 && !(fin(p->u_lo) && fin(p->u_hi) && p->u_lo < p->u_hi))
        return mfail(NMPC_E_ARG, "an input box needs finite u_lo < u_hi");
    if (p->tau > 0.0 && !(p->u_cold > p->u_lo && p->u_cold < p->u_hi))
        return mfail(NMPC_E_ARG, "u_cold must lie strictly inside the input box");
    if (p->model == NMPC_MODEL_PLATE) {
        if (!p->act) return mfail(NMPC_E_ARG, "the plate model needs the actuator nodes");
        std::vector<char> seen((size_t)p->nsx * p->nsy, 0);
        for (int j = 0; j < p->n_inputs; ++j) {
            const int a = p->act[j];
            if (a < 0 || a >= p->nsx * p->nsy || seen[a])
                return mfail(NMPC_E_ARG, "actuator nodes must be distinct grid nodes");
            seen[a] = 1;
        }
        if (!(fin(p->alpha) && fin(p->beta) && fin(p->rad) && fin(p->t_amb)))
            return mfail(NMPC_E_ARG, "plate constants must be finite");
    } else {
        if (!p->B) return mfail(NMPC_E_ARG, "the heat and wave models need a dense B");
        if (!(fin(p->k0) && fin(p->k1) && fin(p->damp)))
            return mfail(NMPC_E_ARG, "k0, k1, damp must be finite");
    }
    return NMPC_OK;
}

int check_model_options(const nmpc_options *o)
{
    if (!o) return mfail(NMPC_E_ARG, "options are NULL");
    if (!(o->tol >= 0.0) || o->max_iter < 0 || o->n_sweep < 1 || o->n_sweep > 16 ||
        o->n_schur < 0 || o->n_schur > 16)
        return mfail(NMPC_E_ARG, "tol >= 0, max_iter >= 0, 1 <= n_sweep <= 16, 0 <= n_schur <= 16");
    if (o->upper < NMPC_UPPER_JACOBI || o->upper > NMPC_UPPER_SGS)
        return mfail(NMPC_E_ARG, "unknown upper layer");
    if (o->residual != NMPC_RES_SCALED && o->residual != NMPC_RES_PAPER)
        return mfail(NMPC_E_ARG, "residual must be NMPC_RES_SCALED or NMPC_RES_PAPER");
    if (o->precision != NMPC_FP64)
        return mfail(NMPC_E_UNSUPPORTED, "the model engine sweeps in FP64 only");
    if (o->omega != 1.0) return mfail(NMPC_E_UNSUPPORTED, "the model engine takes omega = 1");
    if (o->xref_per_stage) return mfail(NMPC_E_UNSUPPORTED, "the model engine takes one reference");
    return NMPC_OK;
}

void model_release(nmpc_model *h)
{
    for (void *p : {(void *)h->d_nodeinp, (void *)h->d_act, (void *)h->d_B, (void *)h->d_X[0],
                    (void *)h->d_X[1], (void *)h->d_U[0], (void *)h->d_U[1], (void *)h->d_L[0],
                    (void *)h->d_L[1], (void *)h->d_lim, (void *)h->d_info_d, (void *)h->d_info_i})
        if (p) (void)hipFree(p);
    if (h->t0) (void)hipEventDestroy(h->t0);
    if (h->t1) (void)hipEventDestroy(h->t1);
    delete h;
}

nmpc::ModelArgs model_args(const nmpc_model *h, int count)
{
    nmpc::ModelArgs a{};
    const nmpc_model_problem &p = h->prob;
    a.model = p.model;
    a.neumann = p.boundary == NMPC_BC_NEUMANN;
    a.nsx = p.nsx; a.nsy = p.nsy; a.nodes = h->nodes; a.nxg = h->nxg; a.m = h->m; a.N = h->N;
    a.h = p.h; a.q = p.q; a.qv = p.qv; a.r = p.r; a.gamma = p.gamma;
    a.tau = p.tau; a.ulo = p.u_lo; a.uhi = p.u_hi;
    a.alpha = p.alpha; a.beta = p.beta; a.rad = p.rad; a.tamb = p.t_amb;
    a.k0 = p.k0; a.k1 = p.k1; a.damp = p.damp;
    const double dx = a.neumann ? 1.0 / (p.nsx - 1) : 1.0 / (p.nsx + 1);
    a.idx2 = 1.0 / (dx * dx);
    if (p.nsy > 1) {
        const double dy = a.neumann ? 1.0 / (p.nsy - 1) : 1.0 / (p.nsy + 1);
        a.idy2 = 1.0 / (dy * dy);
    } else {
        a.idy2 = 0.0;
    }
    a.lpp = -2.0 * a.idx2 - 2.0 * a.idy2;
    a.nodeinp = h->d_nodeinp; a.act = h->d_act; a.B = h->d_B;
    for (int q = 0; q < 2; ++q) { a.X[q] = h->d_X[q]; a.U[q] = h->d_U[q]; a.LAM[q] = h->d_L[q]; }
    a.lim = h->d_lim; a.info_i = h->d_info_i; a.info_d = h->d_info_d;
    a.count = count;
    a.tol = h->opt.tol; a.max_iter = h->opt.max_iter;
    a.n_sw = h->opt.n_sweep; a.n_schur = h->opt.n_schur;
    a.upper = h->opt.upper; a.res_paper = h->opt.residual == NMPC_RES_PAPER;
    return a;
}

int launch_model(nmpc_model *h, nmpc::ModelArgs &a, hipStream_t s)
{
    void *args[] = {(void *)&a};
    MODEL_TRY(hipLaunchKernel(nmpc::model_kernel(h->prob.model, h->ppt), dim3(a.count),
                              dim3(h->threads), args, h->lds, s));
    return NMPC_OK;
}

int model_init(nmpc_model *h, const nmpc::ModelArgs &a, const double *wx, const double *wu,
               const double *wl, hipStream_t s)
{
    nmpc::ModelInit w{wx, wu, wl, h->prob.u_cold, h->prob.tau > 0.0 ? 1 : 0};
    void *args[] = {(void *)&a, (void *)&w};
    const size_t tot = (size_t)a.count * h->N * (size_t)h->nxg;
    MODEL_TRY(hipLaunchKernel(nmpc::model_init_kernel(),
                              dim3((unsigned)std::min<size_t>((tot + 255) / 256 + 1, 4096)), dim3(256),
                              args, 0, s));
    return NMPC_OK;
}

}  // namespace

extern "C" {

int nmpc_model_create(const nmpc_model_problem *prob, const nmpc_options *opt, int32_t max_batch,
                      nmpc_model **out)
{
    if (!out) return mfail(NMPC_E_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_model(prob);
    if (rc) return rc;
    nmpc_options o;
    if (opt) o = *opt; else nmpc_default_options(&o);
    rc = check_model_options(&o);
    if (rc) return rc;
    if (max_batch < 1) return mfail(NMPC_E_ARG, "max_batch must be >= 1");
    nmpc_model *h = new (std::nothrow) nmpc_model();
    if (!h) return mfail(NMPC_E_OOM, "host allocation failed");
    h->prob = *prob;
    h->opt = o;
    h->max_batch = max_batch;
    h->nodes = prob->nsx * prob->nsy;
    h->nxg = prob->model == NMPC_MODEL_WAVE ? 2 * h->nodes : h->nodes;
    h->m = prob->n_inputs;
    h->N = prob->horizon;
    // one node per thread up to 1024 nodes; beyond, 4 or 8 nodes per thread
    // on at most 512 threads (kernel register budget of 256 VGPRs)
    h->ppt = h->nodes <= 1024 ? 1 : (h->nodes <= 2048 ? 4 : 8);
    h->threads = std::min(h->ppt == 1 ? 1024 : 512, (h->nodes + h->ppt - 1) / h->ppt);
    h->threads = std::max(64, (h->threads + 63) / 64 * 64);
    const int waves = h->threads / 64;
    h->lds = sizeof(double) * (2 * (size_t)h->nodes + 5 * nmpc::kModelMaxM +
                               (size_t)waves * nmpc::kModelMaxM) +
             sizeof(unsigned long long) * 4 * waves;
    h->prob.act = nullptr;
    h->prob.B = nullptr;
    hipError_t e = hipSuccess;
    auto A = [&](void **p, size_t bytes) { if (e == hipSuccess) e = hipMalloc(p, bytes); };
    const size_t sx = (size_t)max_batch * h->N * h->nxg, su = (size_t)max_batch * h->N * h->m;
    for (int q = 0; q < 2; ++q) {
        A((void **)&h->d_X[q], sizeof(double) * sx);
        A((void **)&h->d_L[q], sizeof(double) * sx);
        A((void **)&h->d_U[q], sizeof(double) * su);
    }
    A((void **)&h->d_lim, sizeof(double) * max_batch * h->N);
    A((void **)&h->d_info_d, sizeof(double) * 2 * max_batch);
    A((void **)&h->d_info_i, sizeof(int) * 4 * max_batch);
    if (prob->model == NMPC_MODEL_PLATE) {
        h->act.assign(prob->act, prob->act + h->m);
        h->nodeinp.assign(h->nodes, -1);
        for (int j = 0; j < h->m; ++j) h->nodeinp[h->act[j]] = j;
        A((void **)&h->d_act, sizeof(int) * h->m);
        A((void **)&h->d_nodeinp, sizeof(int) * h->nodes);
        if (e == hipSuccess) e = hipMemcpy(h->d_act, h->act.data(), sizeof(int) * h->m, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(h->d_nodeinp, h->nodeinp.data(), sizeof(int) * h->nodes, hipMemcpyHostToDevice);
    } else {
        A((void **)&h->d_B, sizeof(double) * h->nodes * h->m);
        if (e == hipSuccess)
            e = hipMemcpy(h->d_B, prob->B, sizeof(double) * h->nodes * h->m, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipEventCreate(&h->t0);
    if (e == hipSuccess) e = hipEventCreate(&h->t1);
    if (e == hipSuccess && h->lds > 64 * 1024) {
        for (int ppt : {1, 4, 8})
            if (e == hipSuccess)
                e = hipFuncSetAttribute(nmpc::model_kernel(prob->model, ppt),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds);
    }
    if (e != hipSuccess) {
        const std::string msg = std::string("model engine setup: ") + hipGetErrorString(e);
        const int code = e == hipErrorOutOfMemory ? NMPC_E_OOM : NMPC_E_DEVICE;
        model_release(h);
        return mfail(code, msg);
    }
    *out = h;
    return NMPC_OK;
}

int nmpc_model_set_options(nmpc_model *h, const nmpc_options *opt)
{
    if (!h) return mfail(NMPC_E_ARG, "handle is NULL");
    const int rc = check_model_options(opt);
    if (rc) return rc;
    h->opt = *opt;
    return NMPC_OK;
}

int nmpc_model_solve_batch(nmpc_model *h, int32_t count, const double *x0, const double *xref,
                           const double *warm_x, const double *warm_u, const double *warm_lam,
                           double *out_x, double *out_u, double *out_lam, nmpc_info *info,
                           void *stream)
{
    if (!h) return mfail(NMPC_E_ARG, "handle is NULL");
    if (count < 1 || count > h->max_batch) return mfail(NMPC_E_ARG, "count must be in 1..max_batch");
    if (!x0 || !xref || !out_x || !out_u || !out_lam)
        return mfail(NMPC_E_ARG, "x0, xref and the outputs are required");
    const bool any = warm_x || warm_u || warm_lam, all = warm_x && warm_u && warm_lam;
    if (any && !all) return mfail(NMPC_E_UNSUPPORTED, "the model engine takes cold or (x, u, lambda) starts");
    hipStream_t s = (hipStream_t)stream;
    nmpc::ModelArgs a = model_args(h, count);
    a.x0 = x0; a.xref = xref;
    int rc = model_init(h, a, warm_x, warm_u, warm_lam, s);
    if (rc) return rc;
    a.out_x = out_x; a.out_u = out_u; a.out_lam = out_lam;
    if (h->timing) MODEL_TRY(hipEventRecord(h->t0, s));
    rc = launch_model(h, a, s);
    if (rc) return rc;
    if (h->timing) MODEL_TRY(hipEventRecord(h->t1, s));
    std::vector<int> ii(4 * (size_t)count);
    std::vector<double> dd(2 * (size_t)count);
    MODEL_TRY(hipMemcpyAsync(ii.data(), h->d_info_i, sizeof(int) * 4 * count, hipMemcpyDeviceToHost, s));
    MODEL_TRY(hipMemcpyAsync(dd.data(), h->d_info_d, sizeof(double) * 2 * count, hipMemcpyDeviceToHost, s));
    MODEL_TRY(hipStreamSynchronize(s));
    if (h->timing) {
        float ms = 0.f;
        MODEL_TRY(hipEventElapsedTime(&ms, h->t0, h->t1));
        h->kernel_ms += ms;
        h->launches += 1;
    }
    int worst = NMPC_OK;
    for (int b = 0; b < count; ++b) {
        const int status = ii[4 * b + 1];
        if (h->timing) h->units += (long long)ii[4 * b + 3] * h->N;
        if (info) {
            info[b].r_scaled = dd[2 * b];
            info[b].r_paper = dd[2 * b + 1];
            info[b].iters = ii[4 * b];
            info[b].status = status;
            info[b].fp32_iters = 0;
            info[b].start_used = any ? 1 : 0;
            info[b].err_vs_fp64 = 0.0;
        }
        if (status != NMPC_OK && worst == NMPC_OK) worst = status;
    }
    return worst;
}

int nmpc_model_residual_batch(nmpc_model *h, int32_t count, const double *x0, const double *xref,
                              const double *x, const double *u, const double *lam,
                              double *r_scaled, double *r_paper, void *stream)
{
    if (!h) return mfail(NMPC_E_ARG, "handle is NULL");
    if (count < 1 || count > h->max_batch) return mfail(NMPC_E_ARG, "count must be in 1..max_batch");
    if (!x0 || !xref || !x || !u || !lam || !r_scaled || !r_paper)
        return mfail(NMPC_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    nmpc::ModelArgs a = model_args(h, count);
    a.x0 = x0; a.xref = xref;
    // the trajectory as given (no clipping into the box)
    nmpc::ModelInit w{x, u, lam, 0.0, 0};
    {
        void *args[] = {(void *)&a, (void *)&w};
        const size_t tot = (size_t)count * h->N * (size_t)h->nxg;
        MODEL_TRY(hipLaunchKernel(nmpc::model_init_kernel(),
                                  dim3((unsigned)std::min<size_t>((tot + 255) / 256 + 1, 4096)),
                                  dim3(256), args, 0, s));
    }
    a.residual_only = 1;
    const int rc = launch_model(h, a, s);
    if (rc) return rc;
    std::vector<double> dd(2 * (size_t)count);
    MODEL_TRY(hipMemcpyAsync(dd.data(), h->d_info_d, sizeof(double) * 2 * count, hipMemcpyDeviceToHost, s));
    MODEL_TRY(hipStreamSynchronize(s));
    for (int b = 0; b < count; ++b) {
        r_scaled[b] = dd[2 * b];
        r_paper[b] = dd[2 * b + 1];
    }
    return NMPC_OK;
}

int nmpc_model_timing_enable(nmpc_model *h, int32_t enable)
{
    if (!h) return mfail(NMPC_E_ARG, "handle is NULL");
    h->timing = enable != 0;
    if (h->timing) { h->kernel_ms = 0.0; h->launches = 0; h->units = 0; }
    return NMPC_OK;
}

int nmpc_model_timing_read(const nmpc_model *h, double *kernel_ms, int64_t *launches, int64_t *units)
{
    if (!h) return mfail(NMPC_E_ARG, "handle is NULL");
    if (kernel_ms) *kernel_ms = h->kernel_ms;
    if (launches) *launches = h->launches;
    if (units) *units = h->units;
    return NMPC_OK;
}

void nmpc_model_destroy(nmpc_model *h)
{
    if (h) model_release(h);
}

}  // extern "C"
