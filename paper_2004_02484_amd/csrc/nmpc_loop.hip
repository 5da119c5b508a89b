// nmpc_loop.hip -- closed-loop helpers: the shifted start and the plant step;
// and the gathering of a batch's per-instance results for one host copy.
//
// Shifted start (Remark rmk_gamma reuses the previous step's optimum): the
// previous solution moved one stage ahead, s_i <- s_{i+1}, with the last
// stage repeated. Plant: the model advanced by one explicit-Euler step of
// length dt with the applied input, x+ = x + dt (k(x) .* (L x) + B u), on the
// dense [iy][ix] layout with zero Dirichlet values.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmpc_device.h"

namespace nmpc {

// out_s[b][i] = s[b][min(i + 1, N - 1)] for rows of w values per stage.
__global__ void k_shift(const double *s, double *out, long long count, int N, long long w)
{
    const size_t tot = (size_t)count * N * w, stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
        const size_t b = t / ((size_t)N * w), r = t % ((size_t)N * w);
        const int i = (int)(r / w);
        const size_t p = r % w;
        const int src = i + 1 < N ? i + 1 : N - 1;
        out[t] = s[(b * N + src) * w + p];
    }
}

__global__ void k_plant(const PlantArgs a)
{
    const int n = a.nsx * a.nsy, m = a.lx * a.ly;
    const size_t tot = (size_t)a.count * n, stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
        const size_t b = t / n;
        const int p = (int)(t % n), iy = p / a.nsx, ix = p % a.nsx;
        const double *x = a.x + b * n;
        const double *u = a.u + b * (size_t)a.ldu;
        const double xc = x[p];
        const double l = ix > 0 ? x[p - 1] : 0.0, r = ix + 1 < a.nsx ? x[p + 1] : 0.0;
        double Lx = (l + r - 2.0 * xc) * a.idx2;
        if (a.nsy > 1) {
            const double d = iy > 0 ? x[p - a.nsx] : 0.0, up = iy + 1 < a.nsy ? x[p + a.nsx] : 0.0;
            Lx += (d + up - 2.0 * xc) * a.idy2;
        }
        double Bu = 0.0;
        for (int j = 0; j < m; ++j)
            Bu += a.gy[(j / a.lx) * a.nsy + iy] * a.gx[(j % a.lx) * a.nsx + ix] * u[j];
        a.out[t] = xc + a.dt * (a.k0 * (1.0 + a.k1 * xc) * Lx + Bu);
    }
}

// out[b] = instance b's results (one thread per instance).
__global__ void k_info_pack(const PackArgs a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.count) return;
    InfoPack p;
    p.s[0] = a.st[b];
    p.s[1] = a.st[a.B + b];
    p.rf[0] = a.rfin[2 * b];
    p.rf[1] = a.rfin[2 * b + 1];
    p.du[0] = a.du[2 * b];
    p.du[1] = a.du[2 * b + 1];
    p.iters = a.iters[b];
    p.used = a.start ? a.start[b] : -1;
    a.out[b] = p;
}

const void *info_pack_kernel() { return (const void *)&k_info_pack; }
const void *shift_kernel() { return (const void *)&k_shift; }
const void *plant_kernel() { return (const void *)&k_plant; }

}  // namespace nmpc
