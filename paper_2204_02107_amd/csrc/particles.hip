// Lagrangian particles of Section 2.3: one-way coupled point particles with
// drag and gravity, advanced by implicit Euler in the bound velocity field.
#include "particles.h"

#include <rocprim/device/device_radix_sort.hpp>

namespace dnslab {
namespace {

// Trilinear interpolation of a collocated cell field (cell (i, j, k) at
// (i dx, j dy, k dz), periodic) at one position, in FP64.
template <typename T>
__device__ __forceinline__ double interp3(const T* __restrict__ f, const Grid& g, const int i[2], const int j[2],
                                          const int k[2], const double w[3]) {
    double out = 0.0;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz) {
        const double wz = cz ? w[2] : 1.0 - w[2];
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
            const double wy = cy ? w[1] : 1.0 - w[1];
            const long long row = ((long long)k[cz] * g.ny + j[cy]) * g.nx;
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                const double wx = cx ? w[0] : 1.0 - w[0];
                out += (wx * wy * wz) * (double)f[row + i[cx]];
            }
        }
    }
    return out;
}

// Index of the cell holding position x along an axis of n cells of size d
// (the lower interpolation corner, wrapped periodically).
__device__ __forceinline__ int cell_of(double x, double d, int n) {
    long long i0 = (long long)floor(x / d) % n;
    if (i0 < 0) i0 += n;
    return (int)i0;
}

// Wrap into [0, L) like a floored modulo.
__device__ __forceinline__ double wrap_box(double x, double L) {
    double r = x - L * floor(x / L);
    return r >= L ? r - L : r;
}

template <typename T>
__global__ __launch_bounds__(256) void k_particles(const ParticleArgs<T> a) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.n) return;
    const Grid& g = a.g;
    const double pos[3] = {a.px[q], a.py[q], a.pz[q]};
    const double vel[3] = {a.vx[q], a.vy[q], a.vz[q]};
    const int nn[3] = {g.nx, g.ny, g.nz};
    int lo[3][2];
    double w[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double s = pos[ax] / g.d[ax];
        const double fl = floor(s);
        long long i0 = (long long)fl % nn[ax];
        if (i0 < 0) i0 += nn[ax];
        lo[ax][0] = (int)i0;
        lo[ax][1] = (int)(i0 + 1 == nn[ax] ? 0 : i0 + 1);
        w[ax] = s - fl;
    }
    const double uf[3] = {interp3(a.u, g, lo[0], lo[1], lo[2], w), interp3(a.v, g, lo[0], lo[1], lo[2], w),
                          interp3(a.w, g, lo[0], lo[1], lo[2], w)};
    // drag coefficient from the velocities at the start of the step
    const double rel = sqrt((uf[0] - vel[0]) * (uf[0] - vel[0]) + (uf[1] - vel[1]) * (uf[1] - vel[1]) +
                            (uf[2] - vel[2]) * (uf[2] - vel[2]));
    const double d = a.diam[q];
    const double re = rel * d / a.nu;
    const double cd = 1.0 + pow(re, 2.0 / 3.0) / 6.0;
    const double tp = a.rho_p * d * d / (18.0 * a.rho_f * a.nu);
    const double k = cd / tp;
    const double dt = a.dtp ? *a.dtp : a.dt;
    const double gv[3] = {a.g_acc[0], a.g_acc[1], a.g_acc[2]};
    const double L[3] = {a.box[0], a.box[1], a.box[2]};
    double vn[3], pn[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        vn[ax] = (vel[ax] + dt * k * uf[ax] + dt * gv[ax]) / (1.0 + dt * k);
        pn[ax] = wrap_box(pos[ax] + dt * vn[ax], L[ax]);
    }
    a.px[q] = pn[0]; a.py[q] = pn[1]; a.pz[q] = pn[2];
    a.vx[q] = vn[0]; a.vy[q] = vn[1]; a.vz[q] = vn[2];
}

__global__ __launch_bounds__(256) void k_particle_keys(const double* __restrict__ pos, long long n, Grid g,
                                                       unsigned* __restrict__ keys, unsigned* __restrict__ vals) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int i = cell_of(pos[q], g.d[0], g.nx);
    const int j = cell_of(pos[n + q], g.d[1], g.ny);
    const int k = cell_of(pos[2 * n + q], g.d[2], g.nz);
    keys[q] = (unsigned)i + (unsigned)g.nx * ((unsigned)j + (unsigned)g.ny * (unsigned)k);
    vals[q] = (unsigned)q;
}

// out[q] = in[perm[q]]
__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ in, const unsigned* __restrict__ perm,
                                                long long n, double* __restrict__ out) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) out[q] = in[perm[q]];
}

}  // namespace

template <typename T>
hipError_t launch_particles(const ParticleArgs<T>& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const long long nb = (a.n + 255) / 256;
    hipLaunchKernelGGL((k_particles<T>), dim3((unsigned)nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t particle_sort_bytes(long long n, size_t* bytes) {
    *bytes = 0;
    return rocprim::radix_sort_pairs(nullptr, *bytes, (const unsigned*)nullptr, (unsigned*)nullptr,
                                     (const unsigned*)nullptr, (unsigned*)nullptr, (size_t)n);
}

hipError_t sort_particles(const Grid& g, long long n, double* pos, double* vel, double* diam,
                          const ParticleSortScratch& s, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_particle_keys, dim3(nb), dim3(256), 0, st, pos, n, g, s.keys[0], s.vals[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // cell indices are below nx ny nz < 2^31: sort on the bits that can be set
    unsigned end_bit = 1;
    while (end_bit < 32 && ((unsigned long long)1 << end_bit) < (unsigned long long)g.n) ++end_bit;
    size_t bytes = s.sort_bytes;
    e = rocprim::radix_sort_pairs(s.sort_tmp, bytes, s.keys[0], s.keys[1], s.vals[0], s.vals[1], (size_t)n, 0u,
                                  end_bit, st);
    if (e != hipSuccess) return e;
    double* arrays[7] = {pos, pos + n, pos + 2 * n, vel, vel + n, vel + 2 * n, diam};
    for (double* a : arrays) {
        hipLaunchKernelGGL(k_gather, dim3(nb), dim3(256), 0, st, (const double*)a, (const unsigned*)s.vals[1], n,
                           s.tmp);
        e = hipMemcpyAsync(a, s.tmp, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

template hipError_t launch_particles<double>(const ParticleArgs<double>&, hipStream_t);
template hipError_t launch_particles<float>(const ParticleArgs<float>&, hipStream_t);

}  // namespace dnslab
