// nmpc_net_model.hip -- the warm-start network as one object behind the C ABI
// (nmpc_net_*): parameters, optimizer state and activation buffers on the
// device, the layer sequence of the forward pass, its backward pass and the
// Adam step, and a binary weight format. Every step is a launch of the
// library's network kernels (the nmpc_gemm_* / elementwise entry points) on
// the caller's stream.
//
// Layers, rows = instance x actuator (count * L^2 rows):
//   X  = features(x0, xref)           [rows][K0p]  bf16 (and fp32 for the map)
//   H1 = relu(X W1 + b1)              [rows][H]    fp32 + bf16 copy
//   H2 = relu(H1 W2 + b2)
//   H3 = relu(H2 W3 + b3)
//   Y  = H3 W4 + b4 + X Ws[p]         [rows][N]    Ws[p]: per actuator p, fp32
//   u[b][i][p] = U_SCALE * Y[b L^2 + p][i]
// with hidden = 0 the network is the per-actuator map alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "nmpc.h"
#include "nmpc_net.h"

namespace {

constexpr float kUScale = 4.0f;   // targets are u / 4
constexpr int kKsplit = 8;        // K parts of the per-actuator map
constexpr char kMagic[8] = {'N', 'M', 'P', 'C', 'N', 'E', 'T', '1'};

enum { P_W1, P_B1, P_W2, P_B2, P_W3, P_B3, P_W4, P_B4, P_WS, P_COUNT };
const char *kParamNames[P_COUNT] = {"W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "Ws"};

int nfail(int code, const std::string &msg)
{
    nmpc_set_last_error(msg.c_str());
    return code;
}

#define NET_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return nfail(e_ == hipErrorOutOfMemory ? NMPC_E_OOM : NMPC_E_DEVICE,        \
                         std::string(#expr) + ": " + hipGetErrorString(e_));            \
    } while (0)
#define NET_RC(expr)                      \
    do {                                  \
        const int rc_ = (expr);           \
        if (rc_ != NMPC_OK) return rc_;   \
    } while (0)

// splitmix64: a counter-based generator for the initial weights
uint64_t splitmix(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
double uniform_pm1(uint64_t &s) { return 2.0 * ((splitmix(s) >> 11) * (1.0 / 9007199254740992.0)) - 1.0; }

}  // namespace

struct nmpc_net {
    nmpc_net_config cfg{};
    int m = 0, K0 = 0, K0p = 0, H = 0, N = 0, max_rows = 0;
    int64_t numel[P_COUNT] = {};
    float *w[P_COUNT] = {}, *g[P_COUNT] = {}, *mom[P_COUNT] = {}, *vel[P_COUNT] = {};
    uint16_t *wb[P_COUNT] = {};   // bf16 copies of W1..W4
    // activations [rows][...]
    uint16_t *X = nullptr, *H1b = nullptr, *H2b = nullptr, *H3b = nullptr, *dYb = nullptr;
    uint16_t *dHb[3] = {};
    float *Xf = nullptr, *H1 = nullptr, *H2 = nullptr, *H3 = nullptr, *Y = nullptr, *dY = nullptr;
    float *T = nullptr, *sse = nullptr, *work = nullptr, *dH[3] = {};
    int step = 0;
    std::vector<void *> allocs;
};

namespace {

int net_alloc(nmpc_net *n, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes > 0 ? bytes : 1);
    if (e != hipSuccess)
        return nfail(e == hipErrorOutOfMemory ? NMPC_E_OOM : NMPC_E_DEVICE,
                     std::string("network buffers: ") + hipGetErrorString(e));
    n->allocs.push_back(*p);
    return NMPC_OK;
}

void net_release(nmpc_net *n)
{
    for (void *p : n->allocs) (void)hipFree(p);
    delete n;
}

bool is_matrix(int p) { return p == P_W1 || p == P_W2 || p == P_W3 || p == P_W4; }

int refresh_bf16(nmpc_net *n, hipStream_t s)
{
    for (int p = 0; p < P_COUNT; ++p)
        if (n->wb[p]) NET_RC(nmpc_to_bf16(n->w[p], n->wb[p], n->numel[p], s));
    return NMPC_OK;
}

// Y [rows][N] for `count` instances (device x0, xref [count][ns^2]).
int forward_rows(nmpc_net *n, int count, const double *x0, const double *xref, hipStream_t s,
                 bool keep_xf)
{
    const int rows = count * n->m, H = n->H, N = n->N, K0 = n->K0p, m = n->m;
    // feature rows in HBM: bf16 for the hidden path, fp32 for the map's
    // gradient (the map itself gathers its features in place)
    if (H > 0 || keep_xf)
        NET_RC(nmpc_net_features(x0, xref, count, n->cfg.ns, n->cfg.lattice, n->cfg.win, n->cfg.planes,
                                 keep_xf ? n->Xf : nullptr, H > 0 ? n->X : nullptr, K0, s));
    if (H > 0) {
        // the first layer has few output tiles and a long K: split K so that
        // about 512 workgroups run (the partials fit the workspace: at most
        // 512 tiles of 64 x 64)
        const int tiles = ((H + 63) / 64) * ((rows + 63) / 64);
        const int ks = std::max(1, std::min(8, 512 / tiles));
        NET_RC(nmpc::gemm_bf16_split(0, 0, rows, H, K0, n->X, K0, n->wb[P_W1], H, 0.f, n->H1, H,
                                     n->w[P_B1], 1, n->H1b, H, ks, n->work, s));
        NET_RC(nmpc_gemm_bf16(0, 0, rows, H, H, n->H1b, H, n->wb[P_W2], H, 0.f, n->H2, H, n->w[P_B2], 1,
                              n->H2b, H, s));
        NET_RC(nmpc_gemm_bf16(0, 0, rows, H, H, n->H2b, H, n->wb[P_W3], H, 0.f, n->H3, H, n->w[P_B3], 1,
                              n->H3b, H, s));
        NET_RC(nmpc_gemm_bf16(0, 0, rows, N, H, n->H3b, H, n->wb[P_W4], N, 0.f, n->Y, N, n->w[P_B4], 0,
                              nullptr, 0, s));
    }
    // per-actuator map (rows p, p + m, ... of Y), added to the hidden path's
    // output, or written alone (beta 0) without it
    return nmpc::map_forward(x0, xref, count, n->cfg.ns, n->cfg.lattice, n->cfg.win, n->cfg.planes,
                             n->w[P_WS], K0, N, H > 0 ? 1.f : 0.f, n->Y, n->work, s);
}

}  // namespace

extern "C" {

int nmpc_net_create(const nmpc_net_config *cfg, uint64_t seed, int32_t max_count, nmpc_net **out)
{
    if (!out) return nfail(NMPC_E_ARG, "net_create: out is NULL");
    *out = nullptr;
    if (!cfg || cfg->N < 1 || cfg->ns < 1 || cfg->lattice < 1 || cfg->ns % cfg->lattice ||
        cfg->win < cfg->ns / cfg->lattice || (cfg->win - cfg->ns / cfg->lattice) % 2 ||
        (cfg->planes != 2 && cfg->planes != 5) || cfg->hidden < 0 || max_count < 1)
        return nfail(NMPC_E_ARG, "net_create: bad configuration");
    if (cfg->N > 48 || cfg->lattice > 8)
        return nfail(NMPC_E_UNSUPPORTED, "net_create: the map kernel takes N <= 48 and lattice <= 8");
    nmpc_net *n = new (std::nothrow) nmpc_net();
    if (!n) return nfail(NMPC_E_OOM, "host allocation failed");
    n->cfg = *cfg;
    n->m = cfg->lattice * cfg->lattice;
    n->K0 = cfg->planes * cfg->win * cfg->win + n->m;
    n->K0p = (n->K0 + 31) / 32 * 32;
    n->H = cfg->hidden;
    n->N = cfg->N;
    n->max_rows = max_count * n->m;
    const int64_t K0 = n->K0p, H = n->H, N = n->N, m = n->m;
    const int64_t sizes[P_COUNT] = {K0 * H, H, H * H, H, H * H, H, H * N, H > 0 ? N : 0,
                                    m * K0 * N};
    int rc = NMPC_OK;
    for (int p = 0; p < P_COUNT && !rc; ++p) {
        n->numel[p] = sizes[p];
        const size_t bytes = sizeof(float) * (size_t)sizes[p];
        rc = net_alloc(n, (void **)&n->w[p], bytes);
        if (!rc) rc = net_alloc(n, (void **)&n->g[p], bytes);
        if (!rc) rc = net_alloc(n, (void **)&n->mom[p], bytes);
        if (!rc) rc = net_alloc(n, (void **)&n->vel[p], bytes);
        if (!rc && is_matrix(p)) rc = net_alloc(n, (void **)&n->wb[p], sizeof(uint16_t) * sizes[p]);
    }
    const size_t R = n->max_rows;
    auto A = [&](void **p, size_t bytes) { if (!rc) rc = net_alloc(n, p, bytes); };
    A((void **)&n->X, sizeof(uint16_t) * R * K0);
    A((void **)&n->Xf, sizeof(float) * R * K0);
    A((void **)&n->H1, sizeof(float) * R * H); A((void **)&n->H1b, sizeof(uint16_t) * R * H);
    A((void **)&n->H2, sizeof(float) * R * H); A((void **)&n->H2b, sizeof(uint16_t) * R * H);
    A((void **)&n->H3, sizeof(float) * R * H); A((void **)&n->H3b, sizeof(uint16_t) * R * H);
    A((void **)&n->Y, sizeof(float) * R * N); A((void **)&n->T, sizeof(float) * R * N);
    A((void **)&n->dY, sizeof(float) * R * N); A((void **)&n->dYb, sizeof(uint16_t) * R * N);
    A((void **)&n->sse, sizeof(float) * R);
    // split-K partials: the per-actuator map (up to kKsplit parts of N columns) and
    // the first hidden layer (up to 8 parts of H columns)
    A((void **)&n->work, sizeof(float) * std::max<size_t>((size_t)kKsplit * R * N, (size_t)8 * R * H));
    for (int l = 0; l < 3; ++l) {
        A((void **)&n->dH[l], sizeof(float) * R * H);
        A((void **)&n->dHb[l], sizeof(uint16_t) * R * H);
    }
    if (rc) { net_release(n); return rc; }
    // initial weights: He-uniform hidden layers (W1 rows past the features
    // zero), a small output layer, zero biases and a zero map
    uint64_t st = seed;
    for (int p = 0; p < P_COUNT; ++p) {
        std::vector<float> v((size_t)n->numel[p], 0.f);
        double fan = 0.0, gain = 2.0;
        if (p == P_W1) fan = n->K0;
        if (p == P_W2 || p == P_W3) fan = H;
        if (p == P_W4) { fan = H; gain = 0.1; }
        if (fan > 0.0) {
            const double sc = std::sqrt(3.0 * gain / fan);
            const int64_t cols = p == P_W4 ? N : H;
            for (int64_t t = 0; t < n->numel[p]; ++t) {
                const int64_t row = t / cols;
                v[t] = (p == P_W1 && row >= n->K0) ? 0.f : (float)(uniform_pm1(st) * sc);
            }
        }
        hipError_t e = hipMemcpy(n->w[p], v.data(), sizeof(float) * v.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(n->mom[p], 0, sizeof(float) * v.size());
        if (e == hipSuccess) e = hipMemset(n->vel[p], 0, sizeof(float) * v.size());
        if (e != hipSuccess) { net_release(n); return nfail(NMPC_E_DEVICE, hipGetErrorString(e)); }
    }
    rc = refresh_bf16(n, nullptr);
    if (!rc && hipDeviceSynchronize() != hipSuccess) rc = nfail(NMPC_E_DEVICE, "net_create: init");
    if (rc) { net_release(n); return rc; }
    *out = n;
    return NMPC_OK;
}

int nmpc_net_get(const nmpc_net *n, const char *name, void *host, int64_t count)
{
    if (!n || !name || !host) return nfail(NMPC_E_ARG, "net_get: NULL argument");
    const void *src = nullptr;
    int64_t avail = 0;
    size_t esz = 4;
    for (int p = 0; p < P_COUNT; ++p) {
        if (!std::strcmp(name, kParamNames[p])) { src = n->w[p]; avail = n->numel[p]; }
        if (name[0] == 'g' && !std::strcmp(name + 1, kParamNames[p])) { src = n->g[p]; avail = n->numel[p]; }
    }
    const int64_t R = n->max_rows, H = n->H, N = n->N, K0 = n->K0p;
    struct E { const char *nm; const void *p; int64_t n; size_t es; } tab[] = {
        {"X", n->X, R * K0, 2}, {"Xf", n->Xf, R * K0, 4}, {"H1", n->H1, R * H, 4},
        {"H1b", n->H1b, R * H, 2}, {"H2", n->H2, R * H, 4}, {"H2b", n->H2b, R * H, 2},
        {"H3", n->H3, R * H, 4}, {"H3b", n->H3b, R * H, 2}, {"Y", n->Y, R * N, 4},
        {"T", n->T, R * N, 4}, {"dY", n->dY, R * N, 4}, {"dYb", n->dYb, R * N, 2},
        {"dH1", n->dH[0], R * H, 4}, {"dH1b", n->dHb[0], R * H, 2}, {"dH2", n->dH[1], R * H, 4},
        {"dH2b", n->dHb[1], R * H, 2}, {"dH3", n->dH[2], R * H, 4}, {"dH3b", n->dHb[2], R * H, 2},
        {"Wb1", n->wb[P_W1], n->numel[P_W1], 2}, {"Wb2", n->wb[P_W2], n->numel[P_W2], 2},
        {"Wb3", n->wb[P_W3], n->numel[P_W3], 2}, {"Wb4", n->wb[P_W4], n->numel[P_W4], 2}};
    for (const E &e : tab)
        if (!std::strcmp(name, e.nm)) { src = e.p; avail = e.n; esz = e.es; }
    if (!src) return nfail(NMPC_E_ARG, std::string("net_get: unknown name ") + name);
    if (count < 0 || count > avail) return nfail(NMPC_E_ARG, std::string("net_get: count of ") + name);
    NET_HIP(hipDeviceSynchronize());
    NET_HIP(hipMemcpy(host, src, esz * (size_t)count, hipMemcpyDeviceToHost));
    return NMPC_OK;
}

int nmpc_net_set(nmpc_net *n, const char *name, const float *src, int64_t count, int32_t on_device,
                 void *stream)
{
    if (!n || !name || !src) return nfail(NMPC_E_ARG, "net_set: NULL argument");
    for (int p = 0; p < P_COUNT; ++p)
        if (!std::strcmp(name, kParamNames[p])) {
            if (count != n->numel[p]) return nfail(NMPC_E_ARG, std::string("net_set: size of ") + name);
            hipStream_t s = (hipStream_t)stream;
            NET_HIP(hipMemcpyAsync(n->w[p], src, sizeof(float) * (size_t)count,
                                   on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
            if (n->wb[p]) NET_RC(nmpc_to_bf16(n->w[p], n->wb[p], n->numel[p], s));
            NET_HIP(hipStreamSynchronize(s));
            return NMPC_OK;
        }
    return nfail(NMPC_E_ARG, std::string("net_set: unknown parameter ") + name);
}

int64_t nmpc_net_num_params(const nmpc_net *n)
{
    if (!n) return 0;
    int64_t t = 0;
    for (int p = 0; p < P_COUNT; ++p) t += n->numel[p];
    return t;
}

int nmpc_net_forward(nmpc_net *n, int32_t count, const double *x0, const double *xref, double *u,
                     void *stream)
{
    if (!n || !x0 || !xref || !u) return nfail(NMPC_E_ARG, "net_forward: NULL argument");
    if (count < 1 || count * n->m > n->max_rows) return nfail(NMPC_E_ARG, "net_forward: count");
    hipStream_t s = (hipStream_t)stream;
    NET_RC(forward_rows(n, count, x0, xref, s, false));
    return nmpc_unpack_inputs(n->Y, n->N, count, n->N, n->m, kUScale, u, s);
}

int nmpc_net_backward(nmpc_net *n, int32_t count, const double *x0, const double *xref,
                      const double *u_target, float *loss, void *stream)
{
    if (!n || !x0 || !xref || !u_target) return nfail(NMPC_E_ARG, "net_backward: NULL argument");
    if (count < 1 || count * n->m > n->max_rows) return nfail(NMPC_E_ARG, "net_backward: count");
    hipStream_t s = (hipStream_t)stream;
    const int rows = count * n->m, H = n->H, N = n->N, K0 = n->K0p, m = n->m;
    NET_RC(forward_rows(n, count, x0, xref, s, true));
    NET_RC(nmpc_pack_inputs(u_target, count, N, m, 1.0f / kUScale, n->T, N, s));
    NET_RC(nmpc_mse_grad(n->Y, N, n->T, N, rows, N, 2.0f / ((float)rows * N), n->dY, n->dYb, N,
                         n->sse, s));
    // the per-actuator map (fp32 dY)
    NET_RC(nmpc_gemm_f32(1, K0, N, count, n->Xf, m * K0, K0, n->dY, m * N, N, 0.f, n->g[P_WS], N,
                         (int64_t)K0 * N, m, 1, nullptr, s));
    if (H > 0) {
        NET_RC(nmpc_gemm_bf16(1, 0, H, N, rows, n->H3b, H, n->dYb, N, 0.f, n->g[P_W4], N, nullptr, 0,
                              nullptr, 0, s));
        NET_RC(nmpc_colsum(n->dY, rows, N, N, n->g[P_B4], s));
        // dH_l = (dH_{l+1} W_{l+1}^T) * relu'(H_l), l = 3, 2, 1
        NET_RC(nmpc_gemm_bf16(0, 1, rows, H, N, n->dYb, N, n->wb[P_W4], N, 0.f, n->dH[2], H, nullptr, 0,
                              nullptr, 0, s));
        const uint16_t *hin[3] = {n->X, n->H1b, n->H2b};
        const float *hout[3] = {n->H1, n->H2, n->H3};
        const int wl[3] = {P_W1, P_W2, P_W3}, bl[3] = {P_B1, P_B2, P_B3};
        for (int l = 2; l >= 0; --l) {
            NET_RC(nmpc_relu_grad(n->dH[l], hout[l], n->dHb[l], (int64_t)rows * H, s));
            const int kin = l == 0 ? K0 : H;
            NET_RC(nmpc_gemm_bf16(1, 0, kin, H, rows, hin[l], kin, n->dHb[l], H, 0.f, n->g[wl[l]], H,
                                  nullptr, 0, nullptr, 0, s));
            NET_RC(nmpc_colsum(n->dH[l], rows, H, H, n->g[bl[l]], s));
            if (l > 0)
                NET_RC(nmpc_gemm_bf16(0, 1, rows, H, H, n->dHb[l], H, n->wb[wl[l]], H, 0.f, n->dH[l - 1],
                                      H, nullptr, 0, nullptr, 0, s));
        }
    }
    if (loss) {
        std::vector<float> h(rows);
        NET_HIP(hipMemcpyAsync(h.data(), n->sse, sizeof(float) * rows, hipMemcpyDeviceToHost, s));
        NET_HIP(hipStreamSynchronize(s));
        double t = 0.0;
        for (float v : h) t += v;
        *loss = (float)(t / ((double)rows * N));
    }
    return NMPC_OK;
}

int nmpc_net_adam_step(nmpc_net *n, float lr, float beta1, float beta2, float eps, float weight_decay,
                       uint32_t frozen_mask, void *stream)
{
    if (!n) return nfail(NMPC_E_ARG, "net_adam_step: NULL network");
    ++n->step;
    for (int p = 0; p < P_COUNT; ++p) {
        if ((frozen_mask >> p) & 1u) continue;
        if (n->numel[p] == 0) continue;
        NET_RC(nmpc_adam(n->w[p], n->g[p], n->mom[p], n->vel[p], n->wb[p], n->numel[p], lr, beta1, beta2,
                         eps, p == P_W1 || p == P_W2 || p == P_W3 || p == P_W4 ? weight_decay : 0.f,
                         n->step, (hipStream_t)stream));
    }
    return NMPC_OK;
}

int nmpc_net_train_step(nmpc_net *n, int32_t count, const double *x0, const double *xref,
                        const double *u_target, float lr, float weight_decay, uint32_t frozen_mask,
                        float *loss, void *stream)
{
    NET_RC(nmpc_net_backward(n, count, x0, xref, u_target, loss, stream));
    return nmpc_net_adam_step(n, lr, 0.9f, 0.999f, 1e-8f, weight_decay, frozen_mask, stream);
}

int nmpc_net_save(const nmpc_net *n, const char *path)
{
    if (!n || !path) return nfail(NMPC_E_ARG, "net_save: NULL argument");
    FILE *f = std::fopen(path, "wb");
    if (!f) return nfail(NMPC_E_ARG, std::string("net_save: cannot open ") + path);
    const int32_t hdr[7] = {n->cfg.N, n->cfg.ns, n->cfg.lattice, n->cfg.win, n->cfg.hidden,
                            n->cfg.planes, n->step};
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int32_t), 7, f) == 7;
    for (int p = 0; p < P_COUNT && ok; ++p) {
        std::vector<float> v((size_t)n->numel[p]);
        ok = hipMemcpy(v.data(), n->w[p], sizeof(float) * v.size(), hipMemcpyDeviceToHost) == hipSuccess;
        ok = ok && std::fwrite(v.data(), sizeof(float), v.size(), f) == v.size();
    }
    ok = (std::fclose(f) == 0) && ok;
    return ok ? NMPC_OK : nfail(NMPC_E_DEVICE, std::string("net_save: write failed: ") + path);
}

int nmpc_net_load(nmpc_net *n, const char *path)
{
    if (!n || !path) return nfail(NMPC_E_ARG, "net_load: NULL argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return nfail(NMPC_E_ARG, std::string("net_load: cannot open ") + path);
    char mg[8];
    int32_t hdr[7];
    bool ok = std::fread(mg, 1, 8, f) == 8 && !std::memcmp(mg, kMagic, 8) &&
              std::fread(hdr, sizeof(int32_t), 7, f) == 7;
    ok = ok && hdr[0] == n->cfg.N && hdr[1] == n->cfg.ns && hdr[2] == n->cfg.lattice &&
         hdr[3] == n->cfg.win && hdr[4] == n->cfg.hidden && hdr[5] == n->cfg.planes;
    if (!ok) {
        std::fclose(f);
        return nfail(NMPC_E_ARG, "net_load: not a weight file of this configuration");
    }
    for (int p = 0; p < P_COUNT && ok; ++p) {
        std::vector<float> v((size_t)n->numel[p]);
        ok = std::fread(v.data(), sizeof(float), v.size(), f) == v.size();
        ok = ok && hipMemcpy(n->w[p], v.data(), sizeof(float) * v.size(), hipMemcpyHostToDevice) == hipSuccess;
    }
    std::fclose(f);
    if (!ok) return nfail(NMPC_E_ARG, "net_load: truncated file");
    n->step = hdr[6];
    return refresh_bf16(n, nullptr);
}

void nmpc_net_destroy(nmpc_net *n)
{
    if (n) net_release(n);
}

}  // extern "C"
