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

// Force of the fluid on the solid cells inside an index box (pressure and
// viscous parts, per unit density), and the step's time, into out[0..7].
template <typename T>
struct ForceArgs {
    const T* vel[3];
    const T* p;
    const uint8_t* flags;
    Grid g;
    int box[6];                   // i0, i1, j0, j1, k0, k1
    double nu;
    const StepScalars* sc;        // t and the dt p belongs to
    double* out;                  // Fp (3), Fv (3), t, dt
};

template <typename T>
hipError_t launch_histogram(const HistArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_body_force(const ForceArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_accumulate(const AccArgs<T>& a, hipStream_t s);

}  // namespace dnslab
