// Internal definitions shared by the HIP translation units of libdnslab.
// gfx950 only: 64-wide wavefronts, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <vector>

namespace dnslab {

// Per-cell flag byte (the library's own copy of the mask beta, Section 2.1).
enum : uint8_t {
    F_FLUID = 1,       // beta = 1
    F_FORCED = 2,      // cell is in the sparse forcing list (S > 0)
    F_NEAR_SOLID = 4,  // some face neighbour is solid: div((1-beta) grad p) may be nonzero here
    F_ROOM = 8,        // inside the region of the room-mean diagnostic
};

template <typename T>
struct alignas(2 * sizeof(T)) C2 {
    T x, y;
};

// Grid geometry passed by value to every stencil kernel.
struct Grid {
    int nx, ny, nz;
    long long nxy, n;
    double d[3];       // spacing
    double inv2d[3];   // 1 / (2 dx_a)
    double inv4d[3];   // 1 / (4 dx_a)
    double invd2[3];   // 1 / dx_a^2
    double dv;         // cell volume
};

// Cells next to a solid, where the immersed-boundary term div((1-beta) grad p)
// can be nonzero (Section 2.2), with the solid face neighbours as bits
// (+x, -x, +y, -y, +z, -z) = (1, 2, 4, 8, 16, 32).
struct IBList {
    const int* idx;
    const uint8_t* mask;
    int n;
};

// Scalars of the running step, resident in device memory so that an adaptive
// dt never needs a host round trip.
struct StepScalars {
    double dt;        // time step of the next step
    double rate;      // max_cells sum_a |u_a|/dx_a of the current velocity
    double t;         // simulated time
    long long step;   // steps taken
    double dt_fixed, cfl, rate_floor;
    double last_dt;   // time step of the step just taken (the scalar transport of that step uses it)
    double last_rate; // rate of the velocity that step started from
    int nonfinite;    // sticky flag: the Courant rate was NaN/Inf
    int nonfinite_diag;   // sticky flag: a diagnostic was NaN/Inf
};

// One diagnostics record, same layout as dnslab_diag.
struct DiagRec {
    double t, dt, ke, div_l2, co2_mass, co2_room_mean, cfl_max;
    long long step;
};

// Per-block partial results of the fused reductions (accumulated in registers).
struct Partial {
    double ke, mass, room_num, room_den, rate;   // rate: max
    double div2;
};

// The partials in memory, field-major: field f of block b at p[f * stride + b],
// so that the single-block reductions read each field with coalesced loads.
// Different kernels own different fields: the velocity ones (kinetic energy,
// Courant rate), the scalar ones (CO2 mass and room sums) and the divergence.
enum PartField { PF_KE = 0, PF_RATE, PF_MASS, PF_RNUM, PF_RDEN, PF_DIV2, PF_COUNT };
enum : int {
    PM_VEL = (1 << PF_KE) | (1 << PF_RATE),
    PM_RATE = 1 << PF_RATE,
    PM_SCA = (1 << PF_MASS) | (1 << PF_RNUM) | (1 << PF_RDEN),
    PM_DIV = 1 << PF_DIV2,
};
struct PartSoA {
    double* p;
    int stride;
};

// Sparse forcing list (Section 2.1 source term), sorted by cell index.
struct Forcing {
    const long long* idx;
    const double* S;
    const double* uset;   // 3 per entry
    const double* cset;
    int n;
    double inv_tau;
};

// Block coordinates of a launch: the block's index in its own (per-scenario)
// grid and that grid's dimensions.  A plain launch takes them from blockIdx and
// gridDim; a batched launch over several scenarios derives them from a table.
struct BlockIdx3 {
    unsigned hw;          // linear block index within the scenario's grid
    unsigned gx, gy, gz;  // the scenario's grid dimensions
};

// XCD-aware order for one-dimensional grids: workgroups are dealt to the 8
// XCDs round-robin by hardware id, so consecutive ids would land in
// different L2s; the remap gives each XCD a contiguous range of logical
// blocks (a permutation of [0, nb)).
__device__ __forceinline__ unsigned xcd_block(unsigned hw, unsigned nb) {
    const unsigned x = hw & 7u, q = hw >> 3;
    const unsigned per = nb >> 3, rem = nb & 7u;
    return x * per + min(x, rem) + q;
}

__device__ __forceinline__ BlockIdx3 hw_block() {
    BlockIdx3 b;
    b.gx = gridDim.x;
    b.gy = gridDim.y;
    b.gz = gridDim.z;
    b.hw = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    return b;
}

// One entry of a batched launch table: a kernel's arguments for one scenario
// and that scenario's grid dimensions.
template <class A>
struct BRec {
    A a;
    unsigned g[3];
};

// Scenario of this block in a batched launch: starts[s] <= blockIdx.x < starts[s+1].
__device__ __forceinline__ int batch_slot(const unsigned* __restrict__ starts, int ns) {
    int lo = 0, hi = ns - 1;
    const unsigned b = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Kernel kinds of the step sequence (for recording and batched replay).
enum KernelKind : int {
    KK_MOM = 1, KK_SCA, KK_FILT, KK_CORR, KK_DIV, KK_REFRES, KK_REFCORR, KK_ADVANCE, KK_DIAG,   // stencil.hip
    KK_MOMPAIR, KK_SCAPAIR,
    KK_IB = 32, KK_FXF, KK_FXI, KK_COLS,                                              // fft.hip
};
__host__ __device__ constexpr int kind_code(int base, int mode, int fp32) { return (base << 8) | (mode << 1) | fp32; }

// A launch captured instead of issued: the pool records each scenario's step
// once and replays every position of the sequence as one batched launch.
struct LaunchRecord {
    int kind;             // kind_code(...)
    dim3 grid, block;
    size_t lds;
    std::vector<unsigned char> rec;   // bytes of one BRec<Args>
};
struct Recorder {
    std::vector<LaunchRecord> recs;
};

template <class A>
inline void record_launch(Recorder* r, int kind, dim3 grid, dim3 block, size_t lds, const A& a) {
    BRec<A> b;
    std::memset(&b, 0, sizeof(b));
    b.a = a;
    b.g[0] = grid.x;
    b.g[1] = grid.y;
    b.g[2] = grid.z;
    LaunchRecord lr;
    lr.kind = kind;
    lr.grid = grid;
    lr.block = block;
    lr.lds = lds;
    lr.rec.resize(sizeof(b));
    std::memcpy(lr.rec.data(), &b, sizeof(b));
    r->recs.push_back(std::move(lr));
}

__device__ __forceinline__ int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// Index of cell `cell` in the sorted forcing list (only called for flagged cells).
__device__ __forceinline__ int forced_entry(const Forcing& f, long long cell) {
    int lo = 0, hi = f.n - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (f.idx[mid] < cell) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Wavefront (64 lanes) sum and max with a fixed reduction tree.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide deterministic reduction of the fields MASK of a Partial; the
// block's result goes to slot idx of out (blockDim.x*y*z <= 1024).
template <int MASK>
__device__ inline void block_reduce_partial(Partial p, PartSoA out, int idx) {
    __shared__ double sh[16][PF_COUNT];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthr = blockDim.x * blockDim.y * blockDim.z;
    const int lane = tid & 63, wid = tid >> 6;
    double v[PF_COUNT] = {p.ke, p.rate, p.mass, p.room_num, p.room_den, p.div2};
#pragma unroll
    for (int f = 0; f < PF_COUNT; ++f) {
        if (!(MASK & (1 << f))) continue;
        v[f] = f == PF_RATE ? wave_max(v[f]) : wave_sum(v[f]);
        if (lane == 0) sh[wid][f] = v[f];
    }
    __syncthreads();
    if (tid < PF_COUNT && (MASK & (1 << tid))) {
        const int f = tid;
        const int nw = (nthr + 63) >> 6;
        double r = sh[0][f];
        for (int w = 1; w < nw; ++w) r = f == PF_RATE ? fmax(r, sh[w][f]) : r + sh[w][f];
        out.p[(size_t)f * out.stride + idx] = r;
    }
}

}  // namespace dnslab
