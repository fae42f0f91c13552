// Lagrangian particles of Section 2.3: one-way coupled point particles with
// drag and gravity, advanced by implicit Euler in the bound velocity field.
#include "particles.h"

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

// ---------------------------------------------------------------------------
// Stable least-significant-digit radix sort of (key, value) pairs, 8-bit
// digits.  One pass per digit: every block counts the digits of its chunk of
// SORT_CHUNK consecutive keys (counts stored digit-major: digit d of block b
// at d * nblocks + b), an exclusive scan of those counts gives each (digit,
// block) its first output slot, and every block scatters its chunk in input
// order, each key going after the keys of its digit that precede it (in
// earlier blocks, earlier tiles of its own chunk, earlier waves of its tile,
// earlier lanes of its wave).  Stable passes make the whole sort stable.
// ---------------------------------------------------------------------------
constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 16;
constexpr int SORT_CHUNK = SORT_THREADS * SORT_ITEMS;    // keys per block
constexpr int SORT_RADIX = 256;
constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_CHUNK = SCAN_THREADS * SCAN_ITEMS;   // counts per scan block

__global__ __launch_bounds__(SORT_THREADS) void k_sort_hist(const unsigned* __restrict__ keys, long long n,
                                                             int shift, unsigned* __restrict__ counts, int nblocks) {
    __shared__ unsigned hist[SORT_RADIX];
    const int t = threadIdx.x;
    hist[t] = 0;
    __syncthreads();
    const long long c0 = (long long)blockIdx.x * SORT_CHUNK;
#pragma unroll
    for (int it = 0; it < SORT_ITEMS; ++it) {
        const long long q = c0 + (long long)it * SORT_THREADS + t;
        if (q < n) atomicAdd(&hist[(keys[q] >> shift) & (SORT_RADIX - 1)], 1u);
    }
    __syncthreads();
    counts[(size_t)t * nblocks + blockIdx.x] = hist[t];
}

// Exclusive scan of len values in place, in blocks of SCAN_CHUNK; each block
// writes its total to sums[blockIdx.x].
__device__ __forceinline__ unsigned block_exclusive_scan(unsigned v, unsigned* sh, unsigned& total) {
    // Hillis-Steele over the block's threads in LDS
    const int t = threadIdx.x, nt = blockDim.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        const unsigned add = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    total = sh[nt - 1];
    const unsigned incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_blocks(unsigned* __restrict__ a, long long len,
                                                              unsigned* __restrict__ sums) {
    __shared__ unsigned sh[SCAN_THREADS];
    const long long base = (long long)blockIdx.x * SCAN_CHUNK + (long long)threadIdx.x * SCAN_ITEMS;
    unsigned v[SCAN_ITEMS], run = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = base + i < len ? a[base + i] : 0u;
        run += v[i];
    }
    unsigned total;
    unsigned pre = block_exclusive_scan(run, sh, total);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < len) a[base + i] = pre;
        pre += v[i];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of the block totals (at most SCAN_CHUNK of them) in one block.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(unsigned* __restrict__ sums, int nsums) {
    __shared__ unsigned sh[SCAN_THREADS];
    const int base = threadIdx.x * SCAN_ITEMS;
    unsigned v[SCAN_ITEMS], run = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = base + i < nsums ? sums[base + i] : 0u;
        run += v[i];
    }
    unsigned total;
    unsigned pre = block_exclusive_scan(run, sh, total);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < nsums) sums[base + i] = pre;
        pre += v[i];
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_add(unsigned* __restrict__ a, long long len,
                                                           const unsigned* __restrict__ sums) {
    const unsigned add = sums[blockIdx.x];
    const long long base = (long long)blockIdx.x * SCAN_CHUNK + (long long)threadIdx.x * SCAN_ITEMS;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < len) a[base + i] += add;
}

__global__ __launch_bounds__(SORT_THREADS) void k_sort_scatter(const unsigned* __restrict__ kin,
                                                                const unsigned* __restrict__ vin, long long n,
                                                                int shift, const unsigned* __restrict__ offsets,
                                                                int nblocks, unsigned* __restrict__ kout,
                                                                unsigned* __restrict__ vout) {
    constexpr int NW = SORT_THREADS / 64;
    __shared__ unsigned base[SORT_RADIX];          // next output slot of each digit for this block
    __shared__ unsigned wcnt[NW][SORT_RADIX];      // keys of each digit in each wave of the tile
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    base[t] = offsets[(size_t)t * nblocks + blockIdx.x];
    const long long c0 = (long long)blockIdx.x * SORT_CHUNK;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int it = 0; it < SORT_ITEMS; ++it) {
        const long long q = c0 + (long long)it * SORT_THREADS + t;
        const bool valid = q < n;
        unsigned key = 0, val = 0;
        if (valid) { key = kin[q]; val = vin[q]; }
        // digits 0..255; 256 marks an empty slot (it matches only other empty slots)
        const unsigned d = valid ? (key >> shift) & (SORT_RADIX - 1) : (unsigned)SORT_RADIX;
#pragma unroll
        for (int w = 0; w < NW; ++w) wcnt[w][t] = 0;
        __syncthreads();
        // lanes of this wave holding the same digit
        unsigned long long peers = ~0ull;
#pragma unroll
        for (int b = 0; b < 9; ++b) {
            const unsigned long long m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const unsigned rank = (unsigned)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][d] = (unsigned)__popcll(peers);
        __syncthreads();
        // keys of each digit in earlier waves of the tile
        unsigned before = 0;
        if (valid)
            for (int w = 0; w < wave; ++w) before += wcnt[w][d];
        if (valid) {
            const unsigned dst = base[d] + before + rank;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
        {
            unsigned tot = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) tot += wcnt[w][t];
            base[t] += tot;
        }
        __syncthreads();
    }
}

}  // namespace

long long particle_sort_max() { return (long long)SCAN_CHUNK * SCAN_CHUNK / SORT_RADIX * SORT_CHUNK; }

hipError_t particle_sort_bytes(long long n, size_t* bytes) {
    const long long nblocks = (n + SORT_CHUNK - 1) / SORT_CHUNK;
    const long long len = nblocks * SORT_RADIX;
    const long long nscan = (len + SCAN_CHUNK - 1) / SCAN_CHUNK;
    *bytes = (size_t)(len + nscan + 64) * sizeof(unsigned);
    return hipSuccess;
}

template <typename T>
hipError_t launch_particles(const ParticleArgs<T>& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const long long nb = (a.n + 255) / 256;
    hipLaunchKernelGGL((k_particles<T>), dim3((unsigned)nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t sort_particles(const Grid& g, long long n, double* pos, double* vel, double* diam,
                          const ParticleSortScratch& s, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (n > particle_sort_max()) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_particle_keys, dim3(nb), dim3(256), 0, st, pos, n, g, s.keys[0], s.vals[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // cell indices are below nx ny nz < 2^31: sort on the bits that can be set
    unsigned end_bit = 1;
    while (end_bit < 32 && ((unsigned long long)1 << end_bit) < (unsigned long long)g.n) ++end_bit;
    const int nblocks = (int)((n + SORT_CHUNK - 1) / SORT_CHUNK);
    const long long len = (long long)nblocks * SORT_RADIX;
    const int nscan = (int)((len + SCAN_CHUNK - 1) / SCAN_CHUNK);
    unsigned* counts = (unsigned*)s.sort_tmp;
    unsigned* sums = counts + len;
    int cur = 0;
    for (unsigned shift = 0; shift < end_bit; shift += 8) {
        hipLaunchKernelGGL(k_sort_hist, dim3(nblocks), dim3(SORT_THREADS), 0, st, (const unsigned*)s.keys[cur], n,
                           (int)shift, counts, nblocks);
        hipLaunchKernelGGL(k_scan_blocks, dim3(nscan), dim3(SCAN_THREADS), 0, st, counts, len, sums);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_THREADS), 0, st, sums, nscan);
        hipLaunchKernelGGL(k_scan_add, dim3(nscan), dim3(SCAN_THREADS), 0, st, counts, len, (const unsigned*)sums);
        hipLaunchKernelGGL(k_sort_scatter, dim3(nblocks), dim3(SORT_THREADS), 0, st, (const unsigned*)s.keys[cur],
                           (const unsigned*)s.vals[cur], n, (int)shift, (const unsigned*)counts, nblocks,
                           s.keys[cur ^ 1], s.vals[cur ^ 1]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        cur ^= 1;
    }
    double* arrays[7] = {pos, pos + n, pos + 2 * n, vel, vel + n, vel + 2 * n, diam};
    for (double* a : arrays) {
        hipLaunchKernelGGL(k_gather, dim3(nb), dim3(256), 0, st, (const double*)a, (const unsigned*)s.vals[cur], n,
                           s.tmp);
        e = hipMemcpyAsync(a, s.tmp, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

template hipError_t launch_particles<double>(const ParticleArgs<double>&, hipStream_t);
template hipError_t launch_particles<float>(const ParticleArgs<float>&, hipStream_t);

}  // namespace dnslab
