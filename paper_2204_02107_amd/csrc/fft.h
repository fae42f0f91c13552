// Launch interface of the FFT Poisson kernels (fft.hip).
#pragma once
#include "common.h"

namespace dnslab {

constexpr int FFT_MAX_PASSES = 16;

// Stockham plan of one complex transform length n = prod(rad): passes of
// radix 8, 4, 2 (largest first) then 3.
struct AxisPlan {
    int n;
    int npass;
    int rad[FFT_MAX_PASSES];
    int tpl;        // threads per line = n / rad[0] (1 if n == 1)
};

// Spectrum layouts (complex):
//  - row-major (ps == 0): row (kx = 0..nx/2) stride sx elements, rows ordered
//    (ky, kz) with ky fastest: element (kx, ky, kz) at kx + sx*(ky + ny*kz);
//  - plane-major (ps > 0), used when a whole (ky, kz) plane fits one block:
//    element (kx, ky, kz) at kx*ps + ky + ny*kz with ps = ny*nz.
template <typename T>
struct FFTArgs {
    Grid g;
    int m;              // nx/2 (complex length along x)
    int sx;             // padded row stride of the spectrum (row-major)
    int ps;             // plane stride (plane-major), 0 for row-major
    C2<T>* spec;
    AxisPlan px, py, pz;
    const C2<T>* wx;    // W_m^j, j < m
    const C2<T>* wy;    // W_ny^j
    const C2<T>* wz;    // W_nz^j
    const C2<T>* tw;    // e^{-2 pi i k / nx}, k <= m
    const double* sx2;  // sin^2(2 pi m / N)/dx^2 tables, exact zeros at m = 0, N/2
    const double* sy2;
    const double* sz2;
    double inv_ntot;
    // x pass
    int xtw_lds;        // 1: the W_m and twist tables are staged in each block's LDS; 0: read through the caches
    int nl_x;           // lines per block (power of two)
    int ls_x;           // LDS line stride (complex values, >= m + 1)
    // y / z passes
    int lg_tx_y, lg_tx_z;
    int col_pipe;       // pipelined column passes: -1 where each block gets two tiles or more, 0 never, 1 wherever they apply
    // fused plane pass: lines per LDS chunk of the y and the z transforms
    int lg_ca, lg_cb;
};

// Fused plane pass: complex values held in registers per thread, and the
// block size for ny (a multiple of ny, at most YZ_THREADS).  1024-thread
// blocks (four waves per SIMD) hide the LDS and barrier latency of the one
// block per plane; that leaves 128 registers per thread, enough for planes of
// 8192 FP64 or 16384 FP32 values.
#ifndef DNSLAB_YZ_THREADS32
#define DNSLAB_YZ_THREADS32 1024
#endif
#ifndef DNSLAB_YZ_THREADS64
#define DNSLAB_YZ_THREADS64 1024
#endif
constexpr int YZ_THREADS = DNSLAB_YZ_THREADS64;     // FP64
constexpr int YZ_THREADS32 = DNSLAB_YZ_THREADS32;   // FP32
// Values per thread of the kernel instances: the smallest that holds the plane
// is used, since the larger ones need more registers (FP64 with 8 spills a few).
// FP64: 4, 6, 8 (planes up to 8192 values); FP32: 4, 8, 12, 16 (up to 16384).
// The FP64 table repeats its last entry so that both have YZ_NQ_MAX entries.
constexpr int YZ_NQ_MAX = 4;
constexpr int YZ_QS64[YZ_NQ_MAX] = {4, 6, 8, 8};
constexpr int YZ_QS32[YZ_NQ_MAX] = {4, 8, 12, 16};
constexpr int YZ_NQ64 = 3;
constexpr int YZ_NQ32 = 4;
template <typename T>
constexpr int yz_q(int i) { return sizeof(T) == 8 ? YZ_QS64[i] : YZ_QS32[i]; }
inline int yz_threads(int ny, bool fp32 = false) {
    const int cap = fp32 ? YZ_THREADS32 : YZ_THREADS;
    return ny > cap ? 0 : ny * (cap / ny);
}
// Index into YZ_QS of the instance for a plane of `plane` values on nthr
// threads, -1 if no instance holds it.
inline int yz_instance(bool fp32, int nthr, long long plane) {
    const int nq = fp32 ? YZ_NQ32 : YZ_NQ64;
    for (int i = 0; i < nq; ++i)
        if ((long long)(fp32 ? YZ_QS32[i] : YZ_QS64[i]) * nthr >= plane) return i;
    return -1;
}

// Arguments of the kernels that take more than the FFT description.
template <typename T>
struct IbArgs {
    IBList ib;
    Grid g;
    const T* p;
    T* r;
    T* r0s;
    int first;
};
template <typename T>
struct FxfArgs {
    FFTArgs<T> f;
    const T* r;
};
template <typename T>
struct FxiArgs {
    FFTArgs<T> f;
    T* p;
};

// Every launch_* issues one kernel on stream s, or, when rec is non-NULL,
// records it for batched replay without issuing it.

// r = r0 + div((1-beta) grad p) at the listed cells, in place in r.  On the
// first iteration (first != 0) r holds r0 and r0 is saved into r0s[e];
// later iterations read r0 from r0s.
template <typename T>
hipError_t launch_ib_rhs(const IBList& ib, const Grid& g, const T* p, T* r, T* r0s, int first, hipStream_t s,
                         Recorder* rec = nullptr);

// Forward x pass: real-to-complex along x of r into the spectrum.
template <typename T>
hipError_t launch_fft_x_fwd(const FFTArgs<T>& a, const T* r, hipStream_t s, Recorder* rec = nullptr);
template <typename T>
hipError_t launch_fft_y(const FFTArgs<T>& a, bool inverse, hipStream_t s, Recorder* rec = nullptr);
// z pass: forward, divide by lambda * ntot (zero on the null modes), inverse.
template <typename T>
hipError_t launch_fft_z_solve(const FFTArgs<T>& a, hipStream_t s, Recorder* rec = nullptr);
// Plane-major layout only: y forward, z solve and y inverse of each kx plane
// in one block (one read and one write of the spectrum).
template <typename T>
hipError_t launch_fft_yz_solve(const FFTArgs<T>& a, hipStream_t s, Recorder* rec = nullptr);
// Inverse x pass: C2R along x into p.
template <typename T>
hipError_t launch_fft_x_inv(const FFTArgs<T>& a, T* p, hipStream_t s, Recorder* rec = nullptr);

// The twiddle tables (W_m^j, W_ny^j, W_nz^j, e^{-2 pi i k/nx} for k <= m, in
// that order, contiguous at w) and the symbol tables (sin^2(2 pi j/N)/dx^2 for
// x (j <= m), y, z, contiguous at s2) of grid g, computed on the device; the
// same layout as the tables a context uploads.
template <typename T>
hipError_t launch_fft_tables(C2<T>* w, double* s2, const Grid& g, hipStream_t s);

// Batched replay of one recorded FFT-kernel position (see launch_batched_stencil).
hipError_t launch_batched_fft(int kind, const void* tab, const unsigned* starts, int ns, unsigned total_blocks,
                              dim3 block, size_t lds, hipStream_t s);

AxisPlan make_axis_plan(int n);

}  // namespace dnslab
