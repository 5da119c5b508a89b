// nmpc_gs.hip -- Gauss-Seidel upper layers (Sec. 4.4, Jacobi-type variants):
// forward (eq. fgs), backward, and symmetric (eq. sgs: a backward sweep, then
// a forward sweep, both with the regularization reference u~ = u^k).
//
// A sweep visits the stages in order and solves each stage block from the
// current trajectory, in which the stages visited before already hold their
// new values, so the stages of one instance are sequential. One workgroup
// therefore owns one instance for the whole solve (a persistent launch with one
// workgroup per instance): it keeps the input-factor tables in LDS, walks the
// stages with the same fused stage code as the Jacobi kernel, and takes its
// convergence decisions itself, without host polling.
//
// Buffers: S^j lives in buffer j & 1. The first sweep of an iteration reads
// S^j and writes buffer (j + 1) & 1, so S^j survives until the residual of
// S^j (accumulated during that sweep) has been tested; the residual of S^j
// uses the old neighbour values, the update the new ones. The second sweep of
// SGS works in place in buffer (j + 1) & 1.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "nmpc_device.h"
#include "nmpc_stage.h"

namespace nmpc {

// One sweep over the stages of instance b (dir > 0 forward). res: accumulate
// the residual of the source iterate into acc; res_only: residual only.
template <typename T, int CX, int RY, int LX, int LY>
__device__ __forceinline__ void gs_sweep(const IterArgs &a, Ctx &c, int b, int dir, int src,
                                         int dst, int utb, bool res, bool res_only,
                                         unsigned long long (&acc)[2], bool redo = false)
{
    const int N = a.P.N, n = a.P.n, M = LX * LY;
    StageLoc v{};
    v.so = (long long)b * N * n;
    v.uo = (long long)b * N * M;
    v.xo = (long long)b * n;
    v.src = src;
    v.dst = dst;
    v.utb = utb;
    v.res_at = res ? -1 : -2;
    v.res_only = res_only;
    v.omega = a.omega;
    v.du_at = redo && a.du ? b : -1;
    // forward: x_{i-1} updated (dst), lambda_{i+1} not yet (src); backward:
    // the reverse. The residual of S^j takes both from src.
    v.xpb = dir > 0 ? dst : src;
    v.lnb = dir > 0 ? src : dst;
    v.xrb = src;
    v.lrb = src;
    v.pf = a.gs_pf != 0;
    v.pnb = -1;
    if (v.pf) {   // the sweep's first stage; each stage then prefetches the next
        // the previous sweep's last stage may have just written this stage,
        // and a wave's transfer covers other waves' points: their stores
        // complete before the barrier
        __syncthreads();
        const size_t s0 = (size_t)v.so + (size_t)(dir > 0 ? 0 : N - 1) * n;
        prefetch_xl(c, a.X[src] + s0, a.LAM[src] + s0, n);
    }
    for (int t = 0; t < N; ++t) {
        const int i = dir > 0 ? t : N - 1 - t;
        v.i = i;
        v.last = i == N - 1;
        v.xro = (long long)b * a.xref_inst_stride + (long long)i * a.xref_stage_stride;
        // input box: every stage records the limit of its step for the cut
        v.box_at = a.P.tau > 0.0 && !res_only ? (long long)b * N + i : -1;
        if (v.pf) {
            // the stages ahead are not written in this sweep before they are
            // visited (x_{i+d}, lambda_{i+d} of buffer src)
            v.pnb = t + 1 < N ? src : -1;
            v.pni = i + dir;
            __builtin_amdgcn_s_waitcnt(0);   // this wave's transfers have landed
            __syncthreads();                 // and every other wave's
        }
        stage_body<T, CX, RY, LX, LY>(a, a.P, v, c, acc);
    }
}

// Input box: the fraction-to-the-boundary rule (eq. eq_alphamax) cuts each
// sweep, S <- S + alpha (S_sweep - S), alpha the minimum of the stages' limits
// written during the sweep. out = base + alpha (other - base) over the
// instance's whole trajectory (out is base or other).
__device__ double gs_alpha(const IterArgs &a, Ctx &c, int b)
{
    __syncthreads();   // every stage's limit and every stage's update are written
    double *red = lds_ptr<double>(c, c.off.red);
    double l = 1.0;
    for (int i = c.tid; i < a.P.N; i += c.W * kWave) l = fmin(l, a.apart[(size_t)b * a.P.N + i]);
    red[c.tid] = l;
    __syncthreads();
    double al = 1.0;
    for (int t = 0; t < c.W * kWave && t < a.P.N; ++t) al = fmin(al, red[t]);
    __syncthreads();
    return al;
}

__device__ void gs_blend(const IterArgs &a, Ctx &c, int b, int base, int other, int out,
                         double alpha)
{
    const size_t nx = (size_t)a.P.N * a.P.n, nu = (size_t)a.P.N * a.P.m;
    const size_t xo = (size_t)b * nx, uo = (size_t)b * nu;
    for (size_t t = c.tid; t < nx; t += (size_t)c.W * kWave) {
        const double xb = a.X[base][xo + t], lb = a.LAM[base][xo + t];
        a.X[out][xo + t] = xb + alpha * (a.X[other][xo + t] - xb);
        a.LAM[out][xo + t] = lb + alpha * (a.LAM[other][xo + t] - lb);
    }
    for (size_t t = c.tid; t < nu; t += (size_t)c.W * kWave) {
        const double ub = a.U[base][uo + t];
        a.U[out][uo + t] = ub + alpha * (a.U[other][uo + t] - ub);
    }
    __syncthreads();
}

// upper: kUpperFgs, kUpperBgs or kUpperSgs. The FP32 kernel runs an instance's
// FP32-sweep iterations until its test passes at S^j (mode -> kModeFp64Redo);
// the FP64 kernel then takes one FP64 correction sweep from S^j (the first
// sweep of the variant's iteration), checks the result with a residual-only
// pass and returns it if the test passes, else continues with FP64
// iterations. With a.fp32_finish the FP32 kernel returns S^j itself.
template <int PREC, int CX, int RY, int WB, int LX, int LY>
__global__ void __launch_bounds__(kWave * WB, 1) k_gs(const IterArgs a, const int upper)
{
    using T = typename std::conditional<PREC == kModeFp32, float, double>::type;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Ctx c;
    c.lds = lds_raw;
    tile_setup<T, CX, RY, LX, LY>(c, a.P);
    const int b = blockIdx.x;
    if (b >= a.units) return;
    InstState s = a.st[b];
    if (s.status != kActive) return;
    if (PREC == kModeFp32 && s.mode != kModeFp32) return;
    load_tables<CX, RY, LX, LY>(c, a.gx, a.gy, a.P.nsx, a.P.nsy);
    unsigned long long *bc = lds_ptr<unsigned long long>(c, c.off.nrm);
    const int dir1 = upper == kUpperFgs ? 1 : -1;   // first sweep of an iteration
    int j = s.j, fin = -1;
    bool check_only = false;
    double rs = 0.0, rp = 0.0;
    const bool box = a.P.tau > 0.0;
    if (PREC == kModeFp64 && s.mode == kModeFp64Redo) {
        unsigned long long none[2] = {0, 0};
        gs_sweep<T, CX, RY, LX, LY>(a, c, b, dir1, j & 1, (j & 1) ^ 1, -1, false, false, none,
                                    true);
        if (box) {
            const double al = gs_alpha(a, c, b);
            if (al < 1.0) gs_blend(a, c, b, j & 1, (j & 1) ^ 1, (j & 1) ^ 1, al);
        }
        ++s.e;
        ++j;
        check_only = true;
    }
    for (;;) {
        const int p = j & 1, q = p ^ 1;
        unsigned long long acc[2] = {0, 0};
        gs_sweep<T, CX, RY, LX, LY>(a, c, b, dir1, p, q, -1, true, check_only, acc);
        ++s.e;
        __syncthreads();
        if (c.tid == 0) { bc[0] = acc[0]; bc[1] = acc[1]; }
        __syncthreads();
        rs = bits2d(bc[0]);
        rp = bits2d(bc[1]);
        __syncthreads();   // bc is reused by the next stage's norms
        const double rt = a.res_paper ? rp : rs;
        if (!(rt <= 1.7976931348623157e308)) { fin = kStatusNonfinite; break; }
        if (rt <= a.tol) {
            if (PREC == kModeFp32 && !a.fp32_finish) { s.mode = kModeFp64Redo; break; }
            fin = kStatusOk;
            break;
        }
        if (j >= a.max_iter) { fin = kStatusNoconv; break; }
        if (check_only) {   // the corrected iterate missed the test: iterate on in FP64
            check_only = false;
            continue;
        }
        if (box) {
            const double al = gs_alpha(a, c, b);
            if (al < 1.0) gs_blend(a, c, b, p, q, q, al);
        }
        if (upper == kUpperSgs) {
            if (box) {
                // with the cut, the forward sweep writes buffer p (S^j is no
                // longer needed; u~ = u^j of each stage is read before that
                // stage is overwritten) and the cut result goes to q
                gs_sweep<T, CX, RY, LX, LY>(a, c, b, 1, q, p, p, false, false, acc);
                const double al = gs_alpha(a, c, b);
                gs_blend(a, c, b, q, p, q, al);
            } else {
                gs_sweep<T, CX, RY, LX, LY>(a, c, b, 1, q, q, p, false, false, acc);
            }
            ++s.e;
        }
        ++j;
        if (PREC == kModeFp32) ++s.f32;
    }
    if (c.tid == 0) {
        s.j = j;
        if (PREC == kModeFp64) s.mode = kModeFp64;
        if (fin >= 0) {
            s.status = fin;
            a.iters[b] = j;
            a.rfin[2 * b] = rs;
            a.rfin[2 * b + 1] = rp;
        }
        a.st[b] = s;
        a.st[a.B + b] = s;
    }
}

// Tile shapes (CX columns x RY rows per lane, at most WB waves): one
// workgroup per instance, so the whole CU is one instance's stage; the
// default keeps 16 waves in flight for grids up to 64 rows.
#define NMPC_GS(P, CX_, RY_, WB_)                                                   \
    if (prec == P && cx == CX_ && (ry == 0 || ry == RY_) && lx == LX_ && ly == LY_) { \
        cfg->cx = CX_; cfg->rows = RY_; cfg->max_waves = WB_;                       \
        return (const void *)&k_gs<P, CX_, RY_, WB_, LX_, LY_>;                      \
    }
#define NMPC_GS_DEFAULTS()                                                          \
    NMPC_GS(kModeFp32, 1, 1, 16) NMPC_GS(kModeFp32, 2, 1, 16)                       \
    NMPC_GS(kModeFp32, 3, 1, 16) NMPC_GS(kModeFp32, 4, 1, 16)                       \
    NMPC_GS(kModeFp32, 6, 3, 8)                                                    \
    NMPC_GS(kModeFp64, 1, 2, 8) NMPC_GS(kModeFp64, 2, 2, 8)                         \
    NMPC_GS(kModeFp64, 3, 2, 8) NMPC_GS(kModeFp64, 4, 2, 8)                         \
    NMPC_GS(kModeFp64, 6, 3, 8)
// the 4 x 4 lattice (Gaussian actuators) needs more registers for B and B^T:
// 16 waves only where the tile still fits 128 VGPRs
#define NMPC_GS_LATTICE4()                                                          \
    NMPC_GS(kModeFp32, 1, 1, 16) NMPC_GS(kModeFp32, 2, 2, 8)                        \
    NMPC_GS(kModeFp32, 3, 2, 8) NMPC_GS(kModeFp32, 4, 2, 8)                         \
    NMPC_GS(kModeFp32, 6, 3, 8)                                                    \
    NMPC_GS(kModeFp64, 1, 2, 8) NMPC_GS(kModeFp64, 2, 2, 8)                         \
    NMPC_GS(kModeFp64, 3, 2, 8) NMPC_GS(kModeFp64, 4, 2, 8)                         \
    NMPC_GS(kModeFp64, 6, 3, 8)                                                    \
    NMPC_GS(kModeFp32, 2, 1, 16) NMPC_GS(kModeFp32, 3, 1, 16)                       \
    NMPC_GS(kModeFp32, 4, 1, 16) NMPC_GS(kModeFp32, 4, 4, 4)                        \
    NMPC_GS(kModeFp64, 4, 1, 16) NMPC_GS(kModeFp64, 4, 4, 4)

const void *gs_kernel(int prec, int cx, int ry, int lx, int ly, TileCfg *cfg)
{
#define LX_ 1
#define LY_ 1
    NMPC_GS_DEFAULTS()
#undef LX_
#undef LY_
#define LX_ 2
#define LY_ 1
    NMPC_GS_DEFAULTS()
#undef LX_
#undef LY_
#define LX_ 2
#define LY_ 2
    NMPC_GS_DEFAULTS()
#undef LX_
#undef LY_
#define LX_ 4
#define LY_ 4
    NMPC_GS_LATTICE4()
#undef LX_
#undef LY_
    return nullptr;
}
#undef NMPC_GS_LATTICE4
#undef NMPC_GS_DEFAULTS
#undef NMPC_GS

}  // namespace nmpc
