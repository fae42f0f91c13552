// On-device post-processing of Sections 3.1.1 and 3.3-3.4: the force on an
// obstacle, the CO2 distribution over the room and running sums of the fields
// for time averages.
#include "postproc.h"

namespace dnslab {
namespace {

// Counts of c per bin over the fluid cells of the room region: each block
// counts its cells in LDS, then adds its counts to the global bins (integer
// atomics: the result does not depend on the order).
template <typename T>
__global__ __launch_bounds__(256) void k_histogram(const HistArgs<T> a) {
    extern __shared__ unsigned int hcount[];
    for (int b = threadIdx.x; b < a.nbins; b += blockDim.x) hcount[b] = 0u;
    __syncthreads();
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
         i += (long long)gridDim.x * blockDim.x) {
        const uint8_t fl = a.flags[i];
        if ((fl & F_FLUID) && (fl & F_ROOM)) {
            const double x = floor(((double)a.c[i] - a.lo) / (a.hi - a.lo) * (double)a.nbins);
            if (x == x) {   // a NaN belongs to no bin
                const int b = x < 0.0 ? 0 : (x >= (double)(a.nbins - 1) ? a.nbins - 1 : (int)x);
                atomicAdd(&hcount[b], 1u);
            }
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < a.nbins; b += blockDim.x)
        if (hcount[b]) atomicAdd(&a.counts[b], (unsigned long long)hcount[b]);
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// sums[f][i] += field_f[i] in FP64, for the five bound fields.
template <typename T>
__global__ __launch_bounds__(256) void k_accumulate(const AccArgs<T> a) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
         i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int f = 0; f < 5; ++f) a.sums[f * a.n + i] += (double)a.f[f][i];
    }
}

// Force on the obstacle cells of a box (Section 3.1.1, Table 2).  Pressure:
// the central pressure gradient sums to zero over the periodic grid, so the
// momentum it takes from the fluid is what it holds at the solid cells; the
// obstacle's share is -dV sum_s grad P(s) (P = p / dt, the correction
// u = u* - grad p folding dt into p), i.e. face pressures averaged over the
// two cells of each face.  Viscous: every face between an obstacle cell and a
// fluid cell adds the flux nu u_f A / dx_a of the masked second difference
// into the solid cell (zero velocity there).  One block walks the box
// (obstacles are small) and reduces in a fixed order, so the result is
// reproducible bit for bit.
constexpr int FORCE_THREADS = 256;

template <typename T>
__global__ __launch_bounds__(FORCE_THREADS) void k_body_force(const ForceArgs<T> a) {
    const Grid& g = a.g;
    const int bx = a.box[1] - a.box[0], by = a.box[3] - a.box[2], bz = a.box[5] - a.box[4];
    const long long tot = (long long)bx * by * bz;
    const double inv_dt = 1.0 / a.sc->last_dt;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const int nn[3] = {g.nx, g.ny, g.nz};
    for (long long e = threadIdx.x; e < tot; e += FORCE_THREADS) {
        const int c0[3] = {a.box[0] + (int)(e % bx), a.box[2] + (int)((e / bx) % by), a.box[4] + (int)(e / ((long long)bx * by))};
        const long long ic = c0[0] + (long long)g.nx * (c0[1] + (long long)g.ny * c0[2]);
        if (a.flags[ic] & F_FLUID) continue;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const double area = g.dv / g.d[ax];
#pragma unroll
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                int c[3] = {c0[0], c0[1], c0[2]};
                c[ax] += sgn;
                if (c[ax] < 0) c[ax] += nn[ax];
                if (c[ax] >= nn[ax]) c[ax] -= nn[ax];
                const long long f = c[0] + (long long)g.nx * (c[1] + (long long)g.ny * c[2]);
                acc[ax] -= 0.5 * (double)a.p[f] * inv_dt * (double)sgn * area;
                if (!(a.flags[f] & F_FLUID)) continue;
#pragma unroll
                for (int q = 0; q < 3; ++q) acc[3 + q] += a.nu * (double)a.vel[q][f] * area / g.d[ax];
            }
        }
    }
    __shared__ double red[6][FORCE_THREADS];
#pragma unroll
    for (int q = 0; q < 6; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = FORCE_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < 6; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q) a.out[q] = red[q][0];
        a.out[6] = a.sc->t;
        a.out[7] = a.sc->last_dt;
    }
}

}  // namespace

template <typename T>
hipError_t launch_histogram(const HistArgs<T>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3((a.nbins + 255) / 256), dim3(256), 0, s, a.counts, a.nbins);
    const long long nb = std::min<long long>((a.n + 255) / 256, 4096);
    hipLaunchKernelGGL((k_histogram<T>), dim3((unsigned)std::max<long long>(nb, 1)), dim3(256),
                       (size_t)a.nbins * sizeof(unsigned int), s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_accumulate(const AccArgs<T>& a, hipStream_t s) {
    const long long nb = std::min<long long>((a.n + 255) / 256, 8192);
    hipLaunchKernelGGL((k_accumulate<T>), dim3((unsigned)std::max<long long>(nb, 1)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_body_force(const ForceArgs<T>& a, hipStream_t s) {
    hipLaunchKernelGGL((k_body_force<T>), dim3(1), dim3(FORCE_THREADS), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_body_force<double>(const ForceArgs<double>&, hipStream_t);
template hipError_t launch_body_force<float>(const ForceArgs<float>&, hipStream_t);
template hipError_t launch_histogram<double>(const HistArgs<double>&, hipStream_t);
template hipError_t launch_histogram<float>(const HistArgs<float>&, hipStream_t);
template hipError_t launch_accumulate<double>(const AccArgs<double>&, hipStream_t);
template hipError_t launch_accumulate<float>(const AccArgs<float>&, hipStream_t);

}  // namespace dnslab
