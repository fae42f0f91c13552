// Launch interface of the post-processing kernels (postproc.hip).
#pragma once
#include <algorithm>

#include "common.h"

namespace dnslab {

constexpr int HIST_MAX_BINS = 4096;

template <typename T>
struct HistArgs {
    const T* c;
    const uint8_t* flags;
    long long n;
    int nbins;
    double lo, hi;
    unsigned long long* counts;   // nbins device counters (zeroed by the launch)
};

template <typename T>
struct AccArgs {
    const T* f[5];                // u, v, w, p, c
    double* sums;                 // 5 n values, field-major
    long long n;
};

template <typename T>
hipError_t launch_histogram(const HistArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_accumulate(const AccArgs<T>& a, hipStream_t s);

}  // namespace dnslab
