// fields.hip -- density and velocity fields of a domain, computed on the
// device from the in-place population storage (Sec. 2.3: rho = sum_i f_i,
// rho u = sum_i f_i c_i, plus half the fluid force density with forcing).
//
// The moments of a chunk of cells are formed by one kernel into a device
// staging buffer and copied to the caller's host arrays chunk by chunk:
//   psmdem_read_fields          stages through a buffer the library allocates
//                               for the call (the domain's allocator);
//   psmdem_read_fields_noalloc  stages through `scratch`, a file-scope device
//                               array of PSM_SCRATCH_CELLS cells, and allocates
//                               nothing.
#include <math.h>
#include <mutex>

#include "common.h"
#include "domain.h"

// staging of the no-allocation read-out: rho then u (3 per cell) of up to
// PSM_SCRATCH_CELLS cells (4 doubles per cell, 32 MiB); one copy per device,
// held until the process ends, shared by every call on that device
#define PSM_SCRATCH_CELLS (1 << 20)
static __device__ __align__(256) double scratch[4 * PSM_SCRATCH_CELLS];

namespace {

struct FieldArgs {
    const void* f;
    long long N;
    int n[3];
    int periodic[3];
    int odd;
    const double* wall_corr;  // [6 * 19]
    double F[3];              // constant force density
    double kamp;              // Kolmogorov amplitude along kdir, phase along kax
    int kax, kdir;
};

template <typename S>
__device__ inline double load_pop(const S* f, long long idx) {
    return (double)f[idx];
}
template <>
__device__ inline double load_pop<unsigned short>(const unsigned short* f, long long idx) {
    return (double)__uint_as_float(((unsigned)f[idx]) << 16);  // BF16 bits
}

// moments of cells c0 .. c0 + n - 1 into out: rho[n], then u[3 n]
template <typename S>
__global__ __launch_bounds__(256) void k_moments(FieldArgs A, long long c0, long long n, double* out) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const long long c = c0 + j;
    const int nx = A.n[0], ny = A.n[1];
    const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((long long)nx * ny));
    const int xyz[3] = {x, y, z};
    const S* f = (const S*)A.f;
    double r = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll 1
    for (int i = 0; i < 19; ++i) {
        const int ci[3] = {d3q19_cx(i), d3q19_cy(i), d3q19_cz(i)};
        double g;
        if (!A.odd) {
            g = load_pop(f, (long long)i * A.N + c);
        } else {
            // after an odd step the population moving along c_i sits in slot
            // opp(i) of the upstream cell, or, when the upstream link crosses a
            // wall, in the cell's own slot i without the moving-wall term
            int src[3], face = -1;
            for (int a = 0; a < 3; ++a) {
                int v = xyz[a] - ci[a];
                if (v < 0 || v >= A.n[a]) {
                    if (A.periodic[a]) v = v < 0 ? v + A.n[a] : v - A.n[a];
                    else if (face < 0) face = v < 0 ? 2 * a : 2 * a + 1;
                }
                src[a] = v;
            }
            if (face >= 0)
                g = load_pop(f, (long long)i * A.N + c) + A.wall_corr[19 * face + i];
            else
                g = load_pop(f, (long long)d3q19_opp(i) * A.N + src[0] +
                                    (long long)nx * (src[1] + (long long)ny * src[2]));
        }
        const double fi = g + d3q19_w(i);
        r += fi;
        m0 += fi * (double)ci[0];
        m1 += fi * (double)ci[1];
        m2 += fi * (double)ci[2];
    }
    double F[3] = {A.F[0], A.F[1], A.F[2]};
    if (A.kamp != 0.0)
        F[A.kdir] += A.kamp * sin(2.0 * M_PI * ((double)xyz[A.kax] + 0.5) / (double)A.n[A.kax]);
    out[j] = r;
    out[n + 3 * j + 0] = (m0 + 0.5 * F[0]) / r;
    out[n + 3 * j + 1] = (m1 + 0.5 * F[1]) / r;
    out[n + 3 * j + 2] = (m2 + 0.5 * F[2]) / r;
}

FieldArgs field_args(const psmdem_domain* D) {
    FieldArgs A{};
    A.f = D->f;
    A.N = D->N;
    A.n[0] = D->d.nx;
    A.n[1] = D->d.ny;
    A.n[2] = D->d.nz;
    for (int a = 0; a < 3; ++a) {
        A.periodic[a] = D->geo.periodic[a];
        A.F[a] = D->d.body_force[a];
    }
    A.odd = (D->step & 1) != 0;
    A.wall_corr = D->wall_corr_d;
    A.kamp = D->d.kolm_amp;
    A.kax = D->d.kolm_axis;
    A.kdir = D->d.kolm_dir;
    return A;
}

hipError_t launch_moments(const psmdem_domain* D, long long c0, long long n, double* out) {
    const FieldArgs A = field_args(D);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    switch (D->prec) {
        case PSMDEM_FP64: k_moments<double><<<blocks, 256, 0, D->s>>>(A, c0, n, out); break;
        case PSMDEM_FP32: k_moments<float><<<blocks, 256, 0, D->s>>>(A, c0, n, out); break;
        case PSMDEM_BF16_SHIFTED: k_moments<unsigned short><<<blocks, 256, 0, D->s>>>(A, c0, n, out); break;
        default: k_moments<_Float16><<<blocks, 256, 0, D->s>>>(A, c0, n, out); break;
    }
    return hipGetLastError();
}

// every chunk of at most `chunk` cells through the device buffer `stage`
int read_fields_via(psmdem_domain* D, double* stage, long long chunk, double* rho, double* u) {
    for (long long c0 = 0; c0 < D->N; c0 += chunk) {
        const long long n = D->N - c0 < chunk ? D->N - c0 : chunk;
        PSM_CHECK(launch_moments(D, c0, n, stage));
        if (rho)
            PSM_CHECK(hipMemcpyAsync(rho + c0, stage, sizeof(double) * n, hipMemcpyDeviceToHost, D->s));
        if (u)
            PSM_CHECK(hipMemcpyAsync(u + 3 * c0, stage + n, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, D->s));
        PSM_CHECK(hipStreamSynchronize(D->s));
    }
    return 0;
}

// device address of `scratch` per device, taken once with that device current
std::mutex g_scratch_mu;
double* g_scratch[64] = {};

int scratch_of(int dev, double** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= 64) {
        psm_set_error("device %d out of range", dev);
        return PSMDEM_E_INVALID;
    }
    if (!g_scratch[dev]) {
        int cur = -1;
        PSM_CHECK(hipGetDevice(&cur));
        if (cur != dev) PSM_CHECK(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) PSM_CHECK(hipSetDevice(cur));
        if (e != hipSuccess || !p) return psm_hip_fail(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
        g_scratch[dev] = (double*)p;
    }
    *out = g_scratch[dev];
    return 0;
}

}  // namespace

extern "C" psmdem_status psmdem_read_fields(psmdem_domain* d, double* rho, double* u) {
    if (!d) return PSMDEM_E_INVALID;
    const psmdem_status st = psm_sync_flags(d);
    if (psm_read_fails(st)) return st;
    const long long chunk = d->N < (1ll << 22) ? d->N : (1ll << 22);
    const size_t nb = sizeof(double) * 4 * (size_t)chunk;
    double* stage = (double*)d->talloc(nb);
    if (!stage) {
        psm_set_error("device allocation of %zu bytes for the field read-out failed", nb);
        return PSMDEM_E_NOMEM;
    }
    const int rc = read_fields_via(d, stage, chunk, rho, u);
    d->tfree(stage, nb);
    return rc ? (psmdem_status)rc : st;
}

extern "C" psmdem_status psmdem_read_fields_noalloc(psmdem_domain* d, double* rho, double* u) {
    if (!d) return PSMDEM_E_INVALID;
    const psmdem_status st = psm_sync_flags(d);
    if (psm_read_fails(st)) return st;
    double* stage = nullptr;
    if (int rc = scratch_of(d->dev, &stage)) return (psmdem_status)rc;
    if (int rc = read_fields_via(d, stage, PSM_SCRATCH_CELLS, rho, u)) return (psmdem_status)rc;
    return st;
}
