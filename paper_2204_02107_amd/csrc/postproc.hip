// On-device post-processing of Sections 3.3-3.4: the CO2 distribution over
// the room and running sums of the fields for time averages.
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

template hipError_t launch_histogram<double>(const HistArgs<double>&, hipStream_t);
template hipError_t launch_histogram<float>(const HistArgs<float>&, hipStream_t);
template hipError_t launch_accumulate<double>(const AccArgs<double>&, hipStream_t);
template hipError_t launch_accumulate<float>(const AccArgs<float>&, hipStream_t);

}  // namespace dnslab
