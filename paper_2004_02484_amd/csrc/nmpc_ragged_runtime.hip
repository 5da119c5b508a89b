// nmpc_ragged_runtime.hip -- host runtime of ragged batches: per-instance
// layout, XCD-balanced work list, the per-iteration launch loop (captured as a
// graph of check_every launches, FP32 phase then FP64 phase), the workgroup-size
// autotuner and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "nmpc.h"
#include "nmpc_device.h"

using nmpc::InstState;
using nmpc::IterArgs;
using nmpc::RgArgs;
using nmpc::RgClass;

namespace {

int rg_fail(int code, const std::string &msg)
{
    nmpc_set_last_error(msg.c_str());
    return code;
}

#define RG_TRY(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return rg_fail(e_ == hipErrorOutOfMemory ? NMPC_E_OOM : NMPC_E_DEVICE,    \
                           std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

constexpr int kWaveChoices[3] = {8, 12, 16};
constexpr int kMaxClasses = 64;

int cx_of(int nsx)
{
    const int c = (nsx + 15) / 16;
    return c == 5 ? 6 : c;
}

template <typename T>
int grow(T *&p, size_t &cap, size_t need)
{
    if (need <= cap && p) return NMPC_OK;
    if (p) { (void)hipFree(p); p = nullptr; cap = 0; }
    const size_t n = std::max<size_t>(need, 1);
    RG_TRY(hipMalloc((void **)&p, sizeof(T) * n));
    cap = n;
    return NMPC_OK;
}

}  // namespace

struct nmpc_ragged {
    std::vector<nmpc_problem> cls;
    std::vector<std::vector<double>> gx, gy;
    nmpc_options opt{};
    int max_inst = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr, t0 = nullptr, t1 = nullptr;
    // device class tables, one per workgroup size choice
    RgClass *d_cls[3] = {nullptr, nullptr, nullptr};
    bool fits[3][kMaxClasses] = {};
    double *d_g = nullptr;
    // per-instance arrays [max_inst]
    int *d_icls = nullptr;
    long long *d_off = nullptr;   // 6 arrays of max_inst: xoff soff uoff dxoff dsoff ustart
    int2 *d_umap = nullptr; size_t cap_umap = 0;
    double *d_S[2] = {nullptr, nullptr}; size_t cap_S = 0;
    double *d_in = nullptr; size_t cap_in = 0;    // padded x0 | xref
    unsigned long long *d_rst = nullptr; size_t cap_rst = 0;
    InstState *d_st = nullptr;
    int *d_iters = nullptr;
    double *d_rfin = nullptr;
    unsigned long long *d_du = nullptr;   // [B][2] FP64 correction step (max |du|, max |u|)
    double *d_apart = nullptr; size_t cap_apart = 0;   // input box: step limit per stage unit
    int *d_aupd = nullptr;        // input box: [B] 1 + launch index of the last update
    bool box = false;             // some class has an input box
    int *d_ctr = nullptr;
    int *h_poll = nullptr;
    int gen = 0;                  // bumped when a buffer moves (graphs hold pointers)
    // host layout of the current batch
    std::vector<int> h_icls;
    std::vector<long long> h_off;
    std::vector<int2> h_umap;
    std::vector<double> h_cost;   // stage-points of each instance (balancing)
    size_t S_len = 0, in_len = 0, tot_units = 0, tot_dense_x = 0;
    int count = 0;
    // work list of the current batch: one segment (one launch per upper
    // iteration) per tile case present, eight XCD runs of per_xcd units each
    struct Seg {
        int tcase, per_xcd;
        size_t off;   // first entry in h_umap / d_umap
    };
    std::vector<Seg> segs;
    long long wl_sig = 0;         // identifies the work-list shape (graph key)
    // graphs per precision
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    long long gkey[2][8] = {};
    std::map<unsigned long long, int> tuned;   // class-set mask -> waves
    bool timing = false;
    double kernel_ms = 0.0;
    long long launches = 0, units = 0, units_eval = 0;   // units: evaluated and updated

    double *X(int b) const { return d_S[b]; }
    double *L(int b) const { return d_S[b] + S_len; }
    double *U(int b) const { return d_S[b] + 2 * S_len; }
};

namespace {

void rg_release(nmpc_ragged *r)
{
    if (!r) return;
    for (int q = 0; q < 2; ++q) {
        if (r->gexec[q]) (void)hipGraphExecDestroy(r->gexec[q]);
        if (r->graph[q]) (void)hipGraphDestroy(r->graph[q]);
    }
    for (void *p : {(void *)r->d_cls[0], (void *)r->d_cls[1], (void *)r->d_cls[2], (void *)r->d_g,
                    (void *)r->d_icls, (void *)r->d_off, (void *)r->d_umap, (void *)r->d_S[0],
                    (void *)r->d_S[1], (void *)r->d_in, (void *)r->d_rst, (void *)r->d_st,
                    (void *)r->d_iters, (void *)r->d_rfin, (void *)r->d_ctr, (void *)r->d_du,
                    (void *)r->d_apart, (void *)r->d_aupd})
        if (p) (void)hipFree(p);
    if (r->h_poll) (void)hipHostFree(r->h_poll);
    for (hipEvent_t e : {r->ev, r->t0, r->t1})
        if (e) (void)hipEventDestroy(e);
    if (r->stream) (void)hipStreamDestroy(r->stream);
    delete r;
}

int wave_index(int waves)
{
    for (int q = 0; q < 3; ++q)
        if (kWaveChoices[q] == waves) return q;
    return -1;
}

// Workgroup size for the classes in `mask`: the autotuned choice, else the
// first size whose tiles fit every class.
int pick_waves(const nmpc_ragged *r, unsigned long long mask)
{
    auto it = r->tuned.find(mask);
    if (it != r->tuned.end()) return it->second;
    for (int q = 0; q < 3; ++q) {
        bool ok = true;
        for (int c = 0; c < (int)r->cls.size(); ++c)
            if ((mask >> c) & 1ull) ok = ok && r->fits[q][c];
        if (ok) return kWaveChoices[q];
    }
    return -1;
}

// Host layout of a batch: per-instance offsets.
int layout(nmpc_ragged *r, int count, const int32_t *cls, unsigned long long *mask)
{
    const int nc = (int)r->cls.size();
    r->h_icls.assign(cls, cls + count);
    r->h_off.assign(6 * (size_t)r->max_inst, 0);
    r->h_cost.assign(count, 0.0);
    long long xo = 0, so = 0, uo = 0, dxo = 0, dso = 0, us = 0;
    *mask = 0;
    for (int b = 0; b < count; ++b) {
        const int c = cls[b];
        if (c < 0 || c >= nc) return rg_fail(NMPC_E_ARG, "class index out of range");
        *mask |= 1ull << c;
        const nmpc_problem &p = r->cls[c];
        const long long np = (long long)p.nsy * 16 * cx_of(p.nsx), nd = (long long)p.nsx * p.nsy;
        const long long N = p.horizon, m = (long long)p.lx * p.ly;
        r->h_off[0 * (size_t)r->max_inst + b] = xo;
        r->h_off[1 * (size_t)r->max_inst + b] = so;
        r->h_off[2 * (size_t)r->max_inst + b] = uo;
        r->h_off[3 * (size_t)r->max_inst + b] = dxo;
        r->h_off[4 * (size_t)r->max_inst + b] = dso;
        r->h_off[5 * (size_t)r->max_inst + b] = us;
        xo += np; so += N * np; uo += N * m; dxo += nd; dso += N * nd; us += N;
        r->h_cost[b] = (double)N * np;
    }
    r->in_len = (size_t)xo;
    r->S_len = (size_t)so;
    r->tot_units = (size_t)us;
    r->tot_dense_x = (size_t)dso;
    r->count = count;
    return NMPC_OK;
}

// Work list for workgroup size `waves`: the instances grouped by tile case
// (one segment each, in case order), each group assigned longest-first, as
// whole instances, to the eight XCD runs.
int worklist(nmpc_ragged *r, int waves)
{
    std::map<int, std::vector<int>> by_case;
    for (int b = 0; b < r->count; ++b) {
        const nmpc_problem &p = r->cls[r->h_icls[b]];
        const int tc = nmpc::ragged_tile(p.nsx, p.nsy, waves, nullptr, nullptr);
        if (tc < 0) return rg_fail(NMPC_E_UNSUPPORTED, "a class does not fit this workgroup size");
        by_case[tc].push_back(b);
    }
    r->segs.clear();
    r->h_umap.clear();
    long long sig = waves;
    for (auto &kv : by_case) {
        std::vector<int> &order = kv.second;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return r->h_cost[a] > r->h_cost[b]; });
        std::vector<std::vector<int>> bins(8);
        double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        size_t len[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int b : order) {
            const int x = (int)(std::min_element(load, load + 8) - load);
            bins[x].push_back(b);
            load[x] += r->h_cost[b];
            len[x] += r->cls[r->h_icls[b]].horizon;
        }
        nmpc_ragged::Seg sg{kv.first, (int)*std::max_element(len, len + 8), r->h_umap.size()};
        r->h_umap.resize(sg.off + 8 * (size_t)sg.per_xcd, int2{-1, -1});
        for (int x = 0; x < 8; ++x) {
            size_t t = sg.off + (size_t)x * sg.per_xcd;
            for (int b : bins[x])
                for (int i = 0; i < r->cls[r->h_icls[b]].horizon; ++i) r->h_umap[t++] = int2{b, i};
        }
        r->segs.push_back(sg);
        sig = sig * 1000003 + (long long)sg.tcase * 65537 + sg.per_xcd;
    }
    r->wl_sig = sig;
    return NMPC_OK;
}

int ensure_buffers(nmpc_ragged *r)
{
    const size_t S = 3 * r->S_len;   // X | LAM | U (U is shorter; one allocation)
    size_t cap = r->cap_S;
    if (S > cap || !r->d_S[0]) {
        for (int q = 0; q < 2; ++q)
            if (r->d_S[q]) { (void)hipFree(r->d_S[q]); r->d_S[q] = nullptr; }
        r->cap_S = 0;
        RG_TRY(hipMalloc((void **)&r->d_S[0], sizeof(double) * S));
        RG_TRY(hipMalloc((void **)&r->d_S[1], sizeof(double) * S));
        r->cap_S = S;
        ++r->gen;
    }
    const size_t in0 = r->cap_in, rs0 = r->cap_rst, um0 = r->cap_umap;
    int rc = grow(r->d_in, r->cap_in, 2 * r->in_len);
    if (!rc) rc = grow(r->d_rst, r->cap_rst, 6 * r->tot_units);
    if (!rc) rc = grow(r->d_umap, r->cap_umap, r->h_umap.size());
    const size_t ap0 = r->cap_apart;
    if (!rc && r->box) rc = grow(r->d_apart, r->cap_apart, r->tot_units);
    if (rc) return rc;
    if (r->cap_in != in0 || r->cap_rst != rs0 || r->cap_umap != um0 || r->cap_apart != ap0) ++r->gen;
    return NMPC_OK;
}

IterArgs rg_iter_args(const nmpc_ragged *r)
{
    IterArgs a{};
    a.x0 = r->d_in;
    a.xref = r->d_in + r->in_len;
    for (int b = 0; b < 2; ++b) { a.X[b] = r->X(b); a.U[b] = r->U(b); a.LAM[b] = r->L(b); }
    a.rst = r->d_rst;
    a.pst = r->d_rst + 3 * r->tot_units;
    a.rslot = (long long)r->tot_units;
    a.st = r->d_st; a.iters = r->d_iters; a.rfin = r->d_rfin; a.du = r->d_du;
    a.apart = r->d_apart; a.aupd = r->d_aupd;
    a.ctr = r->d_ctr; a.kofs = 0;
    a.B = r->max_inst;
    a.units = 0;       // per launch: 8 * the segment's per_xcd
    a.per_xcd = 0;
    a.tol = r->opt.tol; a.max_iter = r->opt.max_iter;
    a.n_sw = r->opt.n_sweep; a.n_schur = r->opt.n_schur;
    a.res_paper = r->opt.residual == NMPC_RES_PAPER;
    return a;
}

RgArgs rg_args(const nmpc_ragged *r, int wi)
{
    RgArgs g{};
    const size_t M = r->max_inst;
    g.cls = r->d_cls[wi];
    g.icls = r->d_icls;
    g.xoff = r->d_off;
    g.soff = r->d_off + M;
    g.uoff = r->d_off + 2 * M;
    g.dxoff = r->d_off + 3 * M;
    g.dsoff = r->d_off + 4 * M;
    g.ustart = r->d_off + 5 * M;
    g.umap = r->d_umap;
    g.count = r->count;
    return g;
}

size_t lds_case(int waves, int tcase, int prec)
{
    const int cx[5] = {1, 2, 3, 4, 6};
    return nmpc::lds_layout(4 * waves, waves, cx[tcase / 3], prec == nmpc::kModeFp32 ? 4 : 8, 4, 4,
                            tcase % 3 + 1).total;
}

// One upper iteration: one launch per tile case of the work list.
int launch_rg(nmpc_ragged *r, int prec, int waves, IterArgs a, hipStream_t s)
{
    const int wi = wave_index(waves);
    if (wi < 0) return rg_fail(NMPC_E_UNSUPPORTED, "no ragged kernel for this workgroup size");
    RgArgs g = rg_args(r, wi);
    for (const nmpc_ragged::Seg &sg : r->segs) {
        const void *fn = nmpc::ragged_iterate_kernel(prec, waves, sg.tcase);
        if (!fn) return rg_fail(NMPC_E_UNSUPPORTED, "no ragged kernel for this tile");
        a.units = 8 * sg.per_xcd;
        a.per_xcd = sg.per_xcd;
        g.umap = r->d_umap + sg.off;
        void *args[] = {(void *)&a, (void *)&g};
        const size_t lds = lds_case(waves, sg.tcase, prec);
        if (lds > nmpc::kLdsBytes) return rg_fail(NMPC_E_UNSUPPORTED, "tile exceeds the LDS");
        if (lds > 48 * 1024)
            RG_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        RG_TRY(hipLaunchKernel(fn, dim3(8 * sg.per_xcd), dim3(nmpc::kWave * waves), args, lds, s));
        if (r->box && !a.residual_only)   // input box: the step rule of this case's launch
            RG_TRY(hipLaunchKernel(nmpc::ragged_box_apply_kernel(), dim3(8 * sg.per_xcd), dim3(256),
                                   args, 0, s));
    }
    return NMPC_OK;
}

int ensure_graph(nmpc_ragged *r, int prec, int waves)
{
    const int len = r->opt.check_every;
    // the captured launches hold every pointer and length of the layout
    const long long key[8] = {waves, r->wl_sig, r->count, r->gen, len, (long long)r->in_len,
                              (long long)r->S_len, (long long)r->tot_units};
    if (r->gexec[prec] && std::equal(key, key + 8, r->gkey[prec])) return NMPC_OK;
    if (r->gexec[prec]) { (void)hipGraphExecDestroy(r->gexec[prec]); r->gexec[prec] = nullptr; }
    if (r->graph[prec]) { (void)hipGraphDestroy(r->graph[prec]); r->graph[prec] = nullptr; }
    IterArgs a = rg_iter_args(r);
    RG_TRY(hipStreamBeginCapture(r->stream, hipStreamCaptureModeThreadLocal));
    int rc = NMPC_OK;
    for (int t = 0; t < len && rc == NMPC_OK; ++t) {
        a.kofs = t;
        rc = launch_rg(r, prec, waves, a, r->stream);
    }
    if (rc == NMPC_OK) {
        int *ctr = r->d_ctr;
        int l = len;
        void *args[] = {(void *)&ctr, (void *)&l};
        const hipError_t e = hipLaunchKernel(nmpc::advance_kernel(), dim3(1), dim3(64), args, 0,
                                             r->stream);
        if (e != hipSuccess) rc = rg_fail(NMPC_E_DEVICE, std::string("advance: ") + hipGetErrorString(e));
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(r->stream, &g);
    if (rc != NMPC_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return rg_fail(NMPC_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    r->graph[prec] = g;
    RG_TRY(hipGraphInstantiate(&r->gexec[prec], g, nullptr, nullptr, 0));
    std::copy(key, key + 8, r->gkey[prec]);
    return NMPC_OK;
}

// Layout upload, padded inputs and S^0 of a batch (queued on r->stream after
// the caller's stream).
int prepare(nmpc_ragged *r, int count, const int32_t *cls, const double *x0, const double *xref,
            const double *wx, const double *wu, const double *wl, hipStream_t us, int *waves)
{
    RG_TRY(hipStreamSynchronize(r->stream));   // the host layout arrays are rewritten below
    unsigned long long mask = 0;
    int rc = layout(r, count, cls, &mask);
    if (rc) return rc;
    const int w = *waves > 0 ? *waves : pick_waves(r, mask);
    const int wi = wave_index(w);
    if (wi < 0) return rg_fail(NMPC_E_UNSUPPORTED, "no workgroup size fits every class of the batch");
    for (int c = 0; c < (int)r->cls.size(); ++c)
        if (((mask >> c) & 1ull) && !r->fits[wi][c])
            return rg_fail(NMPC_E_UNSUPPORTED, "a class does not fit this workgroup size");
    *waves = w;
    rc = worklist(r, w);
    if (rc) return rc;
    rc = ensure_buffers(r);
    if (rc) return rc;
    RG_TRY(hipEventRecord(r->ev, us));
    RG_TRY(hipStreamWaitEvent(r->stream, r->ev, 0));
    RG_TRY(hipMemcpyAsync(r->d_icls, r->h_icls.data(), sizeof(int) * count, hipMemcpyHostToDevice, r->stream));
    RG_TRY(hipMemcpyAsync(r->d_off, r->h_off.data(), sizeof(long long) * r->h_off.size(),
                          hipMemcpyHostToDevice, r->stream));
    RG_TRY(hipMemcpyAsync(r->d_umap, r->h_umap.data(), sizeof(int2) * r->h_umap.size(),
                          hipMemcpyHostToDevice, r->stream));
    RgArgs g = rg_args(r, wi);
    {
        double *dst = r->d_in;
        void *args[] = {(void *)&g, (void *)&x0, (void *)&dst};
        RG_TRY(hipLaunchKernel(nmpc::ragged_pad_kernel(), dim3(count), dim3(256), args, 0, r->stream));
        dst = r->d_in + r->in_len;
        void *args2[] = {(void *)&g, (void *)&xref, (void *)&dst};
        RG_TRY(hipLaunchKernel(nmpc::ragged_pad_kernel(), dim3(count), dim3(256), args2, 0, r->stream));
    }
    if (r->box)   // input box: no update recorded for this solve yet (not captured)
        RG_TRY(hipMemsetAsync(r->d_aupd, 0, sizeof(int) * r->max_inst, r->stream));
    IterArgs a = rg_iter_args(r);
    int mode = r->opt.precision == NMPC_FP32_SWEEP ? nmpc::kModeFp32 : nmpc::kModeFp64;
    void *args[] = {(void *)&a, (void *)&g, (void *)&mode, (void *)&wx, (void *)&wu, (void *)&wl};
    RG_TRY(hipLaunchKernel(nmpc::ragged_init_kernel(), dim3(count), dim3(256), args, 0, r->stream));
    return NMPC_OK;
}

int run(nmpc_ragged *r, int waves)
{
    int prec = r->opt.precision == NMPC_FP32_SWEEP ? nmpc::kModeFp32 : nmpc::kModeFp64;
    const long long cap = 2 * ((long long)r->opt.max_iter + 8 + r->opt.check_every);
    long long launched = 0;
    for (;;) {
        int rc = ensure_graph(r, prec, waves);
        if (rc != NMPC_OK) return rc;
        if (r->timing) RG_TRY(hipEventRecord(r->t0, r->stream));
        RG_TRY(hipGraphLaunch(r->gexec[prec], r->stream));
        if (r->timing) RG_TRY(hipEventRecord(r->t1, r->stream));
        launched += r->opt.check_every;
        RG_TRY(hipMemcpyAsync(r->h_poll, r->d_ctr + 2, 2 * sizeof(int), hipMemcpyDeviceToHost, r->stream));
        RG_TRY(hipStreamSynchronize(r->stream));
        if (r->timing) {
            float ms = 0.f;
            RG_TRY(hipEventElapsedTime(&ms, r->t0, r->t1));
            r->kernel_ms += ms;
            r->launches += r->opt.check_every;
        }
        if (r->h_poll[0] >= r->count) break;
        if (prec == nmpc::kModeFp32 && r->h_poll[1] <= 0) prec = nmpc::kModeFp64;
        if (launched > cap)
            return rg_fail(NMPC_E_DEVICE, "instances did not finish within max_iter launches");
    }
    return NMPC_OK;
}

int collect(nmpc_ragged *r, nmpc_info *info)
{
    const int count = r->count;
    std::vector<int> iters(count);
    std::vector<double> rf(2 * (size_t)count);
    std::vector<InstState> st(count), st2(count);
    RG_TRY(hipMemcpyAsync(iters.data(), r->d_iters, sizeof(int) * count, hipMemcpyDeviceToHost, r->stream));
    RG_TRY(hipMemcpyAsync(rf.data(), r->d_rfin, sizeof(double) * 2 * count, hipMemcpyDeviceToHost, r->stream));
    std::vector<unsigned long long> du(2 * (size_t)count);
    RG_TRY(hipMemcpyAsync(du.data(), r->d_du, sizeof(unsigned long long) * 2 * count,
                          hipMemcpyDeviceToHost, r->stream));
    RG_TRY(hipMemcpyAsync(st.data(), r->d_st, sizeof(InstState) * count, hipMemcpyDeviceToHost, r->stream));
    RG_TRY(hipMemcpyAsync(st2.data(), r->d_st + r->max_inst, sizeof(InstState) * count,
                          hipMemcpyDeviceToHost, r->stream));
    RG_TRY(hipStreamSynchronize(r->stream));
    int worst = NMPC_OK;
    for (int b = 0; b < count; ++b) {
        const InstState &s = st[b].status != nmpc::kActive ? st[b] : st2[b];
        if (r->timing) {
            const int eo = nmpc::eval_only_visits(r->opt.precision == NMPC_FP32_SWEEP, false, false, s);
            const long long hz = r->cls[r->h_icls[b]].horizon;
            r->units += (long long)(s.e - eo) * hz;
            r->units_eval += (long long)eo * hz;
        }
        const int status = s.status == nmpc::kActive ? NMPC_E_DEVICE : s.status;
        if (info) {
            info[b].r_scaled = rf[2 * b];
            info[b].r_paper = rf[2 * b + 1];
            info[b].iters = iters[b];
            info[b].status = status;
            info[b].fp32_iters = s.f32;
            info[b].start_used = 0;
            info[b].err_vs_fp64 = nmpc::fp32_step_error(r->opt.precision == NMPC_FP32_SWEEP, false, s,
                                                  &du[2 * b]);
        }
        if (status != NMPC_OK && worst == NMPC_OK) worst = status;
    }
    return worst;
}

int check_class(const nmpc_problem *p)
{
    if (p->dim != 2) return rg_fail(NMPC_E_UNSUPPORTED, "ragged classes are 2D problems");
    if (p->b_kind != NMPC_B_KRON)
        return rg_fail(NMPC_E_UNSUPPORTED, "ragged classes take the Kronecker input form");
    if (p->nsx < 1 || p->nsy < 1 || p->horizon < 1) return rg_fail(NMPC_E_ARG, "sizes must be positive");
    if (p->lx != 4 || p->ly != 4) return rg_fail(NMPC_E_UNSUPPORTED, "ragged classes use the 4 x 4 input lattice");
    if (!p->gx || !p->gy) return rg_fail(NMPC_E_ARG, "gx/gy are NULL");
    if (!(std::isfinite(p->h) && p->h > 0 && std::isfinite(p->r) && p->r > 0 && std::isfinite(p->k0) &&
          std::isfinite(p->k1) && std::isfinite(p->q) && p->q >= 0 && std::isfinite(p->gamma) &&
          p->gamma >= 0))
        return rg_fail(NMPC_E_ARG, "need h > 0, r > 0, q >= 0, gamma >= 0, finite k0, k1");
    for (long long t = 0; t < 4LL * p->nsx; ++t)
        if (!std::isfinite(p->gx[t])) return rg_fail(NMPC_E_ARG, "gx not finite");
    for (long long t = 0; t < 4LL * p->nsy; ++t)
        if (!std::isfinite(p->gy[t])) return rg_fail(NMPC_E_ARG, "gy not finite");
    if (p->nsx > 96 || p->nsy > 96) return rg_fail(NMPC_E_UNSUPPORTED, "ragged classes need nsx, nsy <= 96");
    return NMPC_OK;
}

int check_opts(const nmpc_options *o)
{
    if (!o) return rg_fail(NMPC_E_ARG, "options are NULL");
    if (!(o->tol >= 0.0)) return rg_fail(NMPC_E_ARG, "tol must be >= 0");
    if (o->max_iter < 0 || o->max_iter > 100000000) return rg_fail(NMPC_E_ARG, "bad max_iter");
    if (o->n_sweep < 1 || o->n_sweep > 16) return rg_fail(NMPC_E_ARG, "n_sweep must be 1..16");
    if (o->n_schur < 0 || o->n_schur > 16) return rg_fail(NMPC_E_ARG, "n_schur must be 0..16");
    if (o->precision != NMPC_FP64 && o->precision != NMPC_FP32_SWEEP)
        return rg_fail(NMPC_E_ARG, "unknown precision");
    if (o->check_every < 1 || o->check_every > 4096) return rg_fail(NMPC_E_ARG, "bad check_every");
    if (o->xref_per_stage != 0) return rg_fail(NMPC_E_UNSUPPORTED, "ragged batches take one xref per instance");
    if (o->upper < 0 || o->upper > 3) return rg_fail(NMPC_E_ARG, "unknown upper layer");
    if (o->upper != NMPC_UPPER_JACOBI)
        return rg_fail(NMPC_E_UNSUPPORTED, "ragged batches use the Jacobi upper layer");
    if (o->fp32_finish != 0)
        return rg_fail(NMPC_E_UNSUPPORTED, "ragged batches take the final FP64 correction (fp32_finish 0)");
    return NMPC_OK;
}

int start_ok(const double *wx, const double *wu, const double *wl)
{
    return (!wx && !wu && !wl) || (wx && wu && wl);
}

}  // namespace

extern "C" {

int nmpc_ragged_create(const nmpc_problem *classes, int32_t nclass, const nmpc_options *opt,
                       int32_t max_instances, nmpc_ragged **out)
{
    nmpc_set_last_error("");
    if (!out) return rg_fail(NMPC_E_ARG, "out is NULL");
    *out = nullptr;
    if (!classes || nclass < 1 || nclass > kMaxClasses)
        return rg_fail(NMPC_E_ARG, "need 1..64 classes");
    if (max_instances < 1) return rg_fail(NMPC_E_ARG, "max_instances must be >= 1");
    int rc = check_opts(opt);
    if (rc) return rc;
    for (int c = 0; c < nclass; ++c)
        if ((rc = check_class(&classes[c]))) return rc;
    bool box = false;
    for (int c = 0; c < nclass; ++c) {
        const nmpc_problem &p = classes[c];
        if (!(std::isfinite(p.tau) && p.tau >= 0.0)) return rg_fail(NMPC_E_ARG, "tau must be finite and >= 0");
        if (p.tau > 0.0 && !(std::isfinite(p.u_lo) && std::isfinite(p.u_hi) && p.u_lo < 0.0 &&
                             p.u_hi > 0.0))
            return rg_fail(NMPC_E_ARG, "an input box needs finite u_lo < 0 < u_hi (cold start inside)");
        box = box || p.tau > 0.0;
    }
    nmpc_ragged *r = new (std::nothrow) nmpc_ragged();
    if (!r) return rg_fail(NMPC_E_OOM, "host allocation failed");
    r->opt = *opt;
    r->max_inst = max_instances;
    r->box = box;
    r->cls.assign(classes, classes + nclass);
    r->gx.resize(nclass);
    r->gy.resize(nclass);
    size_t gtot = 0;
    for (int c = 0; c < nclass; ++c) {
        const nmpc_problem &p = classes[c];
        r->gx[c].assign(p.gx, p.gx + 4 * (size_t)p.nsx);
        r->gy[c].assign(p.gy, p.gy + 4 * (size_t)p.nsy);
        r->cls[c].gx = r->gx[c].data();
        r->cls[c].gy = r->gy[c].data();
        gtot += r->gx[c].size() + r->gy[c].size();
    }
    bool any = false;
    for (int q = 0; q < 3; ++q) {
        bool all = true;
        for (int c = 0; c < nclass; ++c) {
            int cx = 0, ry = 0;
            const int w = kWaveChoices[q];
            bool f = nmpc::ragged_tile(classes[c].nsx, classes[c].nsy, w, &cx, &ry) >= 0;
            for (int ts : {4, 8})   // both precisions' layouts within one CU's LDS
                f = f && nmpc::lds_layout(4 * w, w, cx, ts, 4, 4, ry).total <= nmpc::kLdsBytes;
            r->fits[q][c] = f;
            all = all && f;
        }
        any = any || all;
    }
    for (int c = 0; c < nclass; ++c) {
        bool f = false;
        for (int q = 0; q < 3; ++q) f = f || r->fits[q][c];
        if (!f) { rg_release(r); return rg_fail(NMPC_E_UNSUPPORTED, "a class fits no ragged tile"); }
    }
    (void)any;
    hipError_t e = hipSuccess;
    auto A = [&](void **p, size_t bytes) { if (e == hipSuccess) e = hipMalloc(p, bytes); };
    A((void **)&r->d_g, sizeof(double) * gtot);
    for (int q = 0; q < 3; ++q) A((void **)&r->d_cls[q], sizeof(RgClass) * nclass);
    A((void **)&r->d_icls, sizeof(int) * max_instances);
    A((void **)&r->d_off, sizeof(long long) * 6 * max_instances);
    A((void **)&r->d_st, sizeof(InstState) * 2 * max_instances);
    A((void **)&r->d_iters, sizeof(int) * max_instances);
    A((void **)&r->d_rfin, sizeof(double) * 2 * max_instances);
    A((void **)&r->d_du, sizeof(unsigned long long) * 2 * max_instances);
    if (box) A((void **)&r->d_aupd, sizeof(int) * max_instances);
    A((void **)&r->d_ctr, sizeof(int) * 4);
    if (e == hipSuccess) e = hipHostMalloc((void **)&r->h_poll, 2 * sizeof(int), hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&r->t0);
    if (e == hipSuccess) e = hipEventCreate(&r->t1);
    if (e == hipSuccess) e = hipMemset(r->d_ctr, 0, sizeof(int) * 4);
    // class tables
    std::vector<double> g;
    std::vector<RgClass> tab(nclass);
    g.reserve(gtot);
    for (int c = 0; c < nclass && e == hipSuccess; ++c) {
        const nmpc_problem &p = r->cls[c];
        RgClass &k = tab[c];
        const int cx = cx_of(p.nsx);
        k.P.nsx = p.nsx; k.P.nsy = p.nsy; k.P.n = p.nsy * 16 * cx; k.P.N = p.horizon;
        k.P.m = 16; k.P.lx = 4; k.P.ly = 4;
        k.P.h = p.h; k.P.k0 = p.k0; k.P.k1 = p.k1; k.P.q = p.q; k.P.r = p.r; k.P.gamma = p.gamma;
        k.P.tau = p.tau; k.P.ulo = p.u_lo; k.P.uhi = p.u_hi;
        const double dx = 1.0 / (p.nsx + 1), dy = 1.0 / (p.nsy + 1);
        k.P.idx2 = 1.0 / (dx * dx);
        k.P.idy2 = 1.0 / (dy * dy);
        k.P.c0 = 2.0 * k.P.idx2 + 2.0 * k.P.idy2;
        k.gx = r->d_g + g.size();
        g.insert(g.end(), r->gx[c].begin(), r->gx[c].end());
        k.gy = r->d_g + g.size();
        g.insert(g.end(), r->gy[c].begin(), r->gy[c].end());
        k.sx = 16 * cx;
    }
    if (e == hipSuccess) e = hipMemcpy(r->d_g, g.data(), sizeof(double) * g.size(), hipMemcpyHostToDevice);
    for (int q = 0; q < 3 && e == hipSuccess; ++q) {
        for (int c = 0; c < nclass; ++c)
            tab[c].tile = nmpc::ragged_tile(r->cls[c].nsx, r->cls[c].nsy, kWaveChoices[q], nullptr, nullptr);
        e = hipMemcpy(r->d_cls[q], tab.data(), sizeof(RgClass) * nclass, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        rg_release(r);
        return rg_fail(e == hipErrorOutOfMemory ? NMPC_E_OOM : NMPC_E_DEVICE,
                       std::string("ragged create: ") + hipGetErrorString(e));
    }
    *out = r;
    return NMPC_OK;
}

int nmpc_ragged_solve(nmpc_ragged *r, int32_t count, const int32_t *cls, const double *x0,
                      const double *xref, const double *warm_x, const double *warm_u,
                      const double *warm_lam, double *out_x, double *out_u, double *out_lam,
                      nmpc_info *info, void *stream)
{
    nmpc_set_last_error("");
    if (!r || !cls || !x0 || !xref || !out_x || !out_u || !out_lam)
        return rg_fail(NMPC_E_ARG, "NULL argument");
    if (count < 1 || count > r->max_inst) return rg_fail(NMPC_E_ARG, "count outside 1..max_instances");
    if (!start_ok(warm_x, warm_u, warm_lam))
        return rg_fail(NMPC_E_ARG, "a ragged warm start needs all of (x, u, lambda)");
    int waves = 0;
    int rc = prepare(r, count, cls, x0, xref, warm_x, warm_u, warm_lam, (hipStream_t)stream, &waves);
    if (rc) return rc;
    rc = run(r, waves);
    if (rc) return rc;
    {
        IterArgs a = rg_iter_args(r);
        RgArgs g = rg_args(r, wave_index(waves));
        void *args[] = {(void *)&a, (void *)&g, (void *)&out_x, (void *)&out_u, (void *)&out_lam};
        RG_TRY(hipLaunchKernel(nmpc::ragged_output_kernel(), dim3(count), dim3(256), args, 0, r->stream));
    }
    std::vector<nmpc_info> tmp;
    if (!info) { tmp.resize(count); info = tmp.data(); }
    return collect(r, info);
}

int nmpc_ragged_autotune(nmpc_ragged *r, int32_t count, const int32_t *cls, const double *x0,
                         const double *xref, int32_t iters, void *stream, int32_t *waves_out)
{
    nmpc_set_last_error("");
    if (!r || !cls || !x0 || !xref) return rg_fail(NMPC_E_ARG, "NULL argument");
    if (count < 1 || count > r->max_inst) return rg_fail(NMPC_E_ARG, "count outside 1..max_instances");
    if (iters < 1 || iters > 1000) return rg_fail(NMPC_E_ARG, "iters must be 1..1000");
    unsigned long long mask = 0;
    for (int b = 0; b < count; ++b) {
        if (cls[b] < 0 || cls[b] >= (int)r->cls.size()) return rg_fail(NMPC_E_ARG, "class index out of range");
        mask |= 1ull << cls[b];
    }
    const int prec = r->opt.precision == NMPC_FP32_SWEEP ? nmpc::kModeFp32 : nmpc::kModeFp64;
    int best = -1;
    float best_ms = 0.f;
    for (int q = 0; q < 3; ++q) {
        bool ok = true;
        for (int c = 0; c < (int)r->cls.size(); ++c)
            if ((mask >> c) & 1ull) ok = ok && r->fits[q][c];
        if (!ok) continue;
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {   // the first pass loads code and warms caches
            int w = kWaveChoices[q];
            int rc = prepare(r, count, cls, x0, xref, nullptr, nullptr, nullptr, (hipStream_t)stream, &w);
            if (rc) return rc;
            IterArgs a = rg_iter_args(r);
            RG_TRY(hipEventRecord(r->t0, r->stream));
            for (int t = 0; t < iters; ++t) {
                a.kofs = t;
                rc = launch_rg(r, prec, w, a, r->stream);
                if (rc) return rc;
            }
            RG_TRY(hipEventRecord(r->t1, r->stream));
            RG_TRY(hipStreamSynchronize(r->stream));
            RG_TRY(hipEventElapsedTime(&ms, r->t0, r->t1));
        }
        if (best < 0 || ms < best_ms) { best = kWaveChoices[q]; best_ms = ms; }
    }
    if (best < 0) return rg_fail(NMPC_E_UNSUPPORTED, "no workgroup size fits every class of the batch");
    r->tuned[mask] = best;
    if (waves_out) *waves_out = best;
    return NMPC_OK;
}

int nmpc_ragged_config(const nmpc_ragged *r, int32_t count, const int32_t *cls, int32_t *waves)
{
    if (!r || !cls || count < 1) return NMPC_E_ARG;
    unsigned long long mask = 0;
    for (int b = 0; b < count; ++b) {
        if (cls[b] < 0 || cls[b] >= (int)r->cls.size()) return NMPC_E_ARG;
        mask |= 1ull << cls[b];
    }
    const int w = pick_waves(r, mask);
    if (w < 0) return NMPC_E_UNSUPPORTED;
    if (waves) *waves = w;
    return NMPC_OK;
}

int nmpc_ragged_timing_enable(nmpc_ragged *r, int32_t enable)
{
    if (!r) return NMPC_E_ARG;
    RG_TRY(hipStreamSynchronize(r->stream));
    r->timing = enable != 0;
    if (r->timing) { r->kernel_ms = 0.0; r->launches = 0; r->units = 0; r->units_eval = 0; }
    return NMPC_OK;
}

int nmpc_ragged_timing_read(const nmpc_ragged *r, double *kernel_ms, int64_t *launches,
                            int64_t *units)
{
    if (!r) return NMPC_E_ARG;
    if (kernel_ms) *kernel_ms = r->kernel_ms;
    if (launches) *launches = r->launches;
    if (units) *units = r->units;
    return NMPC_OK;
}

int nmpc_ragged_timing_read_eval(const nmpc_ragged *r, int64_t *eval_units)
{
    if (!r) return NMPC_E_ARG;
    if (eval_units) *eval_units = r->units_eval;
    return NMPC_OK;
}

void nmpc_ragged_destroy(nmpc_ragged *r)
{
    if (!r) return;
    (void)hipStreamSynchronize(r->stream);
    rg_release(r);
}

}  // extern "C"
