// Stencil kernels of the projection step (Sections 2.1-2.2), z-marching.
//
// Every kernel maps a thread to one (i, j) column of a block tile and walks a
// chunk of kc cells along z, keeping the z-neighbours of its column in
// registers (a rolling window) so that each z-plane of a field is fetched from
// memory once per chunk.  x- and y-neighbours are loaded directly; within a
// 64-wide wavefront they are the same cache lines as the centre loads, and the
// rows above and below are shared through L1/L2 by the block's other rows.
// All loads and stores are coalesced along x (64 consecutive elements per
// wavefront).
#include "stencil.h"

#include <algorithm>
#include <type_traits>
#include <utility>

namespace dnslab {

namespace {

#ifndef DNSLAB_ZFAST
#define DNSLAB_ZFAST 0
#endif
#ifndef DNSLAB_ZALT
#define DNSLAB_ZALT 1
#endif
#ifndef DNSLAB_FILTER_LDS
#define DNSLAB_FILTER_LDS 1
#endif
#ifndef DNSLAB_FILTER_RING
#define DNSLAB_FILTER_RING 1
#endif
#ifndef DNSLAB_CORRECT_RING
#define DNSLAB_CORRECT_RING 1
#endif
// Prefetch distance, in planes, of the register-ring correction (little
// arithmetic per plane to cover the loads).  Register-ring forms of the
// divergence and of the refinement residual (one cell per thread, 1024-thread
// blocks, no LDS) were measured and dropped: 882 -> 901 us and 809 -> 878 us
// on 1024x512x256.
#ifndef DNSLAB_RING_DIST
#define DNSLAB_RING_DIST 3
#endif
#ifndef DNSLAB_STENCIL_LDS
#define DNSLAB_STENCIL_LDS 1
#endif
constexpr int FILT_LDS = 16;   // filter kind mode bit: LDS-tiled variant
constexpr int FILT_RING = 32;  // filter kind mode bit: LDS-tiled variant with register rings
constexpr int STAGE_LDS = 8;   // RK4 stage kind mode bit: LDS-tiled variant

constexpr double INV_PI6 = 1.0 / (3.14159265358979323846 * 3.14159265358979323846 *
                                  3.14159265358979323846 * 3.14159265358979323846 *
                                  3.14159265358979323846 * 3.14159265358979323846);

struct Col {
    int i, j, im, ip, jm, jp;
    int k0, k1;
    int dir;       // z march direction of the radius-3 filter: +1, or -1 on odd z chunks
    unsigned row, rowm, rowp;   // j*nx, jm*nx, jp*nx
    bool active;
};

// XCD-aware block order.  Workgroups are dealt to the 8 XCDs round-robin by
// hardware id; remapping hardware id -> logical tile so that each XCD owns a
// contiguous range of tiles keeps the y- and z-neighbour rows of a tile in the
// L2 of the XCD that reads them.
__device__ __forceinline__ void logical_block(const BlockIdx3& bi, int& bx, int& by, int& bz) {
    const unsigned gx = bi.gx, gy = bi.gy, gz = bi.gz;
    const unsigned nb = gx * gy * gz;
    const unsigned hw = bi.hw;
    const unsigned x = hw & 7u, q = hw >> 3;
    const unsigned per = nb >> 3, rem = nb & 7u;
    const unsigned L = x * per + min(x, rem) + q;
#if DNSLAB_ZFAST
    bz = (int)(L % gz);
    bx = (int)((L / gz) % gx);
    by = (int)(L / (gz * gx));
#else
    bx = (int)(L % gx);
    by = (int)((L / gx) % gy);
    bz = (int)(L / (gx * gy));
#endif
}

__device__ __forceinline__ Col column(const Grid& g, int kc, const BlockIdx3& bi) {
    Col c;
    int bx, by, bz;
    logical_block(bi, bx, by, bz);
    c.i = bx * blockDim.x + threadIdx.x;
    c.j = by * blockDim.y + threadIdx.y;
    c.k0 = bz * kc;
    c.k1 = min(c.k0 + kc, g.nz);
    // Neighbouring z chunks march towards (or away from) their common
    // boundary at the same time, so the halo planes they both read are
    // fetched once into the L2 instead of twice.
    c.dir = (DNSLAB_ZALT && (bz & 1)) ? -1 : 1;
    c.active = c.i < g.nx && c.j < g.ny;
    if (!c.active) { c.i = 0; c.j = 0; }
    c.im = c.i == 0 ? g.nx - 1 : c.i - 1;
    c.ip = c.i + 1 == g.nx ? 0 : c.i + 1;
    c.jm = c.j == 0 ? g.ny - 1 : c.j - 1;
    c.jp = c.j + 1 == g.ny ? 0 : c.j + 1;
    c.row = (unsigned)c.j * g.nx;
    c.rowm = (unsigned)c.jm * g.nx;
    c.rowp = (unsigned)c.jp * g.nx;
    return c;
}


// Courant rate |u|/dx + |v|/dy + |w|/dz in FP64, summed left to right without
// contraction so that it rounds like a plain sequential evaluation.
__device__ __forceinline__ double courant_rate(double u, double v, double w, const Grid& g) {
#pragma clang fp contract(off)
    double r = fabs(u) / g.d[0];
    r = r + fabs(v) / g.d[1];
    r = r + fabs(w) / g.d[2];
    return r;
}

// ---------------------------------------------------------------------------
// LDS tiles of the z-marching kernels.  A block's tile of one plane (BX x BY
// cells, all inside the grid) is held in LDS with its x and y halo of R cells
// each side (no corners: every stencil here is a sum of one-axis differences),
// as rows of W = BX + 2R values.  The interior comes from the threads' own z
// register windows; halo_map gives each thread its share of the halo.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// The halo cells of this thread (at most HMAX of them) as in-plane source
// offsets and LDS destinations, so that a kernel can load a plane's halo into
// registers one plane ahead of storing it (the rows above and below the tile
// first, then the columns left and right of it).  The launch guarantees
// 2R(BX + BY) <= HMAX * BX * BY.
template <int HMAX>
struct HaloMap {
    unsigned src[HMAX];
    int dst[HMAX];
    int n;
};
template <int R, int HMAX>
__device__ __forceinline__ HaloMap<HMAX> halo_map(int i0, int j0, const Grid& g, int BX, int lgBX, int BY,
                                                  int tid, int nthr) {
    HaloMap<HMAX> hm;
    const int W = BX + 2 * R;
    const int nhy = 2 * R * BX, nh = nhy + 2 * R * BY;
    hm.n = 0;
#pragma unroll
    for (int h = 0; h < HMAX; ++h) {
        const int r = tid + h * nthr;
        hm.src[h] = 0;
        hm.dst[h] = 0;
        if (r < nh) {
            int ly, lx;
            if (r < nhy) {
                const int hr = r >> lgBX;
                ly = hr < R ? hr : BY + hr;
                lx = R + (r - (hr << lgBX));
            } else {
                const int q = r - nhy, row = q / (2 * R), c = q - row * (2 * R);
                ly = R + row;
                lx = c < R ? c : BX + c;
            }
            const int gi = wrap1(i0 + lx - R, g.nx), gj = wrap1(j0 + ly - R, g.ny);
            hm.src[h] = (unsigned)gj * g.nx + gi;
            hm.dst[h] = ly * W + lx;
            hm.n = h + 1;
        }
    }
    return hm;
}

// ---------------------------------------------------------------------------
// Momentum RK4 stage.  k = beta [ -C(u) + nu L u + S (u_set - u)/tau_f + b ]
// with the skew-symmetric convection written per axis as
//   1/2 [D_a(u_a u_i) + u_a D_a u_i] = [(u_a+ + u_a0) u_i+ - (u_a- + u_a0) u_i-] / (4 dx_a).
// ---------------------------------------------------------------------------
template <typename T>
struct MomCoef {
    T q4x, q4y, q4z, ix2, iy2, iz2, nu, b[3];
};
template <typename T>
__device__ __forceinline__ MomCoef<T> mom_coef(const Grid& g, double nu, const double body[3]) {
    MomCoef<T> c;
    c.q4x = T(g.inv4d[0]); c.q4y = T(g.inv4d[1]); c.q4z = T(g.inv4d[2]);
    c.ix2 = T(g.invd2[0]); c.iy2 = T(g.invd2[1]); c.iz2 = T(g.invd2[2]);
    c.nu = T(nu);
    c.b[0] = T(body[0]); c.b[1] = T(body[1]); c.b[2] = T(body[2]);
    return c;
}

// k = F(u) at one cell from its value z0 and its six face neighbours (every
// momentum kernel evaluates F through this one function).
template <typename T>
__device__ __forceinline__ void mom_rhs_cell(const MomCoef<T>& cf, const T z0[3], const T xm[3], const T xp[3],
                                             const T ym[3], const T yp[3], const T zm[3], const T zp[3], uint8_t fl,
                                             const Forcing& frc, unsigned idx, T kv[3]) {
    const T ax_p = xp[0] + z0[0], ax_m = xm[0] + z0[0];
    const T ay_p = yp[1] + z0[1], ay_m = ym[1] + z0[1];
    const T az_p = zp[2] + z0[2], az_m = zm[2] + z0[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T C = (ax_p * xp[c] - ax_m * xm[c]) * cf.q4x + (ay_p * yp[c] - ay_m * ym[c]) * cf.q4y +
                    (az_p * zp[c] - az_m * zm[c]) * cf.q4z;
        const T L = (xp[c] - T(2) * z0[c] + xm[c]) * cf.ix2 + (yp[c] - T(2) * z0[c] + ym[c]) * cf.iy2 +
                    (zp[c] - T(2) * z0[c] + zm[c]) * cf.iz2;
        kv[c] = -C + cf.nu * L + cf.b[c];
    }
    if (fl & F_FORCED) {
        const int e = forced_entry(frc, (long long)idx);
        const T S = T(frc.S[e]) * T(frc.inv_tau);
#pragma unroll
        for (int c = 0; c < 3; ++c) kv[c] += S * (T(frc.uset[3 * e + c]) - z0[c]);
    }
    if (!(fl & F_FLUID)) { kv[0] = T(0); kv[1] = T(0); kv[2] = T(0); }
}

template <typename T, int MODE, bool LDS>
__device__ __forceinline__ void mom_stage_body(const MomArgs<T>& a, const BlockIdx3& bi) {
    const Grid& g = a.g;
    const Col col = column(g, a.kc, bi);
    if (!LDS && !col.active) return;      // the LDS variant only runs on tiles inside the grid
    const int k0 = col.k0, k1 = col.k1;
    const unsigned nxy = (unsigned)g.nxy;
    const T dt = (MODE == ST_RHS) ? T(0) : T(a.dtp ? *a.dtp : a.dt);
    const MomCoef<T> cf = mom_coef<T>(g, a.nu, a.body);
    const T* __restrict__ u0p = a.us[0];
    const T* __restrict__ u1p = a.us[1];
    const T* __restrict__ u2p = a.us[2];
    // LDS tiles (radius 1) of the three stage-input components, two planes
    extern __shared__ unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    const int BX = blockDim.x, BY = blockDim.y, lgBX = __ffs(BX) - 1;
    const int W = BX + 2, tsz = W * (BY + 2);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + BX * ty, nthr = BX * BY;
    const int i0 = col.i - tx, j0 = col.j - ty;
    int buf = 0;
    const unsigned cell = col.row + col.i;
    // LDS variant: loads run one plane ahead of their use (the next z plane
    // of the window, zq, and the next plane's halo, hv)
    constexpr int HM = 2;
    HaloMap<HM> hm;
    T zq[3], hv[3][HM];
    T pa[3] = {T(0), T(0), T(0)}, pn[3] = {T(0), T(0), T(0)};   // acc, u^n of the current plane

    T zm[3], z0[3], zp[3];
    {
        const int km = k0 == 0 ? g.nz - 1 : k0 - 1;
        const unsigned im_ = (unsigned)km * nxy + cell;
        const unsigned i0_ = (unsigned)k0 * nxy + cell;
        zm[0] = u0p[im_]; zm[1] = u1p[im_]; zm[2] = u2p[im_];
        z0[0] = u0p[i0_]; z0[1] = u1p[i0_]; z0[2] = u2p[i0_];
        if (LDS) {
            const unsigned ip_ = (unsigned)wrap(k0 + 1, g.nz) * nxy + cell;
            const unsigned iq_ = (unsigned)wrap(k0 + 2, g.nz) * nxy + cell;
            zp[0] = u0p[ip_]; zp[1] = u1p[ip_]; zp[2] = u2p[ip_];
            zq[0] = u0p[iq_]; zq[1] = u1p[iq_]; zq[2] = u2p[iq_];
            hm = halo_map<1, HM>(i0, j0, g, BX, lgBX, BY, tid, nthr);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (MODE == ST_HALF || MODE == ST_FULL || MODE == ST_LAST) pa[c] = a.acc[c][i0_];
                if (MODE == ST_HALF || MODE == ST_FULL) pn[c] = a.un[c][i0_];
            }
            const unsigned b0 = (unsigned)k0 * nxy;
#pragma unroll
            for (int h = 0; h < HM; ++h) {
                hv[0][h] = h < hm.n ? u0p[b0 + hm.src[h]] : T(0);
                hv[1][h] = h < hm.n ? u1p[b0 + hm.src[h]] : T(0);
                hv[2][h] = h < hm.n ? u2p[b0 + hm.src[h]] : T(0);
            }
        }
    }
    for (int k = k0; k < k1; ++k) {
        const int kp = k + 1 == g.nz ? 0 : k + 1;
        const unsigned base = (unsigned)k * nxy;
        const unsigned idx = base + cell;
        const unsigned ipz = (unsigned)kp * nxy + cell;
        T xm[3], xp[3], ym[3], yp[3];
        if (LDS) {
            T* tb = lds + buf * 3 * tsz;
            buf ^= 1;
            const int ctr = (ty + 1) * W + tx + 1;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                tb[c * tsz + ctr] = z0[c];
#pragma unroll
                for (int h = 0; h < HM; ++h)
                    if (h < hm.n) tb[c * tsz + hm.dst[h]] = hv[c][h];
            }
            if (k + 1 < k1) {
#pragma unroll
                for (int h = 0; h < HM; ++h)
                    if (h < hm.n) {
                        hv[0][h] = u0p[ipz - cell + hm.src[h]];
                        hv[1][h] = u1p[ipz - cell + hm.src[h]];
                        hv[2][h] = u2p[ipz - cell + hm.src[h]];
                    }
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                xm[c] = tb[c * tsz + ctr - 1];
                xp[c] = tb[c * tsz + ctr + 1];
                ym[c] = tb[c * tsz + ctr - W];
                yp[c] = tb[c * tsz + ctr + W];
            }
        } else {
            zp[0] = u0p[ipz]; zp[1] = u1p[ipz]; zp[2] = u2p[ipz];
            const unsigned ixm = base + col.row + col.im, ixp = base + col.row + col.ip;
            const unsigned iym = base + col.rowm + col.i, iyp = base + col.rowp + col.i;
            xm[0] = u0p[ixm]; xm[1] = u1p[ixm]; xm[2] = u2p[ixm];
            xp[0] = u0p[ixp]; xp[1] = u1p[ixp]; xp[2] = u2p[ixp];
            ym[0] = u0p[iym]; ym[1] = u1p[iym]; ym[2] = u2p[iym];
            yp[0] = u0p[iyp]; yp[1] = u1p[iyp]; yp[2] = u2p[iyp];
        }
        const uint8_t fl = a.flags[idx];

        T kv[3];
        mom_rhs_cell<T>(cf, z0, xm, xp, ym, yp, zm, zp, fl, a.frc, idx, kv);

#pragma unroll
        for (int c = 0; c < 3; ++c) {
            // LDS variant: acc and u^n of this cell were loaded one plane ahead
            const T accv = (MODE == ST_HALF || MODE == ST_FULL || MODE == ST_LAST)
                               ? (LDS ? pa[c] : a.acc[c][idx]) : T(0);
            if (MODE == ST_FIRST) {
                a.acc[c][idx] = z0[c] + (dt / T(6)) * kv[c];
                a.out[c][idx] = z0[c] + (dt / T(2)) * kv[c];
            } else if (MODE == ST_HALF || MODE == ST_FULL) {
                const T un = LDS ? pn[c] : a.un[c][idx];
                a.acc[c][idx] = accv + (dt / T(3)) * kv[c];
                a.out[c][idx] = un + (MODE == ST_HALF ? dt / T(2) : dt) * kv[c];
            } else if (MODE == ST_LAST) {
                a.out[c][idx] = accv + (dt / T(6)) * kv[c];
            } else {
                a.out[c][idx] = kv[c];
            }
        }
        if (LDS && k + 1 < k1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (MODE == ST_HALF || MODE == ST_FULL || MODE == ST_LAST) pa[c] = a.acc[c][idx + nxy];
                if (MODE == ST_HALF || MODE == ST_FULL) pn[c] = a.un[c][idx + nxy];
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) { zm[c] = z0[c]; z0[c] = zp[c]; }
        if (LDS) {
#pragma unroll
            for (int c = 0; c < 3; ++c) zp[c] = zq[c];
            if (k + 2 < k1) {
                const unsigned ir_ = (unsigned)wrap(k + 3, g.nz) * nxy + cell;
                zq[0] = u0p[ir_]; zq[1] = u1p[ir_]; zq[2] = u2p[ir_];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Two momentum RK4 stages in one pass (MomPairArgs).  A block owns a BX x BY
// tile and marches along z.  At output plane K it has, in LDS, the stage input
// v of plane K+1 on the tile with a radius-2 halo (and plane K+2 for the z
// neighbours of the ring) and the intermediate stage value w = base + c dt F(v)
// of plane K on the tile with a one-cell ring (no corners); it computes w of
// plane K+1 on tile and ring, then the second stage at plane K on the tile:
//   iteration K:  store v(K+2) -> V;  sync;  w(K+1) on tile + ring -> W;  sync;
//                 F(w) at plane K -> outputs.
// The ring cells (2 BX + 2 BY of them, one per thread from thread 0) keep their
// own z neighbours of v.  Two iterations before the first output plane fill
// the pipeline, so a chunk reads kc + 4 planes of v and evaluates the first
// stage on kc + 2 planes.  Loads run one plane ahead of their use.
// ---------------------------------------------------------------------------
template <int HMAX>
struct PairHalo {
    unsigned src[HMAX];   // in-plane offsets of this thread's halo cells of v
    int dst[HMAX];        // their positions in a V tile
    int n;
};
// Halo of the V tile (row length BX + 4, origin 2): two rows above and below
// the tile spanning x in [-1, BX], two columns left and right spanning the
// tile's rows.  That covers every neighbour of the tile and its ring.
template <int HMAX>
__device__ __forceinline__ PairHalo<HMAX> pair_halo(int i0, int j0, const Grid& g, int BX, int BY, int tid,
                                                    int nthr) {
    PairHalo<HMAX> h;
    const int WV = BX + 4;
    const int rw = BX + 2, nrow = 4 * rw, n = nrow + 4 * BY;
    h.n = 0;
#pragma unroll
    for (int q = 0; q < HMAX; ++q) {
        const int r = tid + q * nthr;
        h.src[q] = 0;
        h.dst[q] = 0;
        if (r < n) {
            int lx, ly;
            if (r < nrow) {
                const int row = r / rw, c = r - row * rw;
                ly = row < 2 ? row - 2 : BY + row - 2;
                lx = c - 1;
            } else {
                const int q2 = r - nrow, row = q2 >> 2, c = q2 & 3;
                ly = row;
                lx = c < 2 ? c - 2 : BX + c - 2;
            }
            const int gi = wrap1(i0 + lx, g.nx), gj = wrap1(j0 + ly, g.ny);
            h.src[q] = (unsigned)gj * g.nx + gi;
            h.dst[q] = (ly + 2) * WV + lx + 2;
            h.n = q + 1;
        }
    }
    return h;
}

// Ring cell r of a BX x BY tile (r < 2 BX + 2 BY): the rows below and above
// the tile, then the columns left and right of it.
__device__ __forceinline__ void ring_cell(int r, int BX, int BY, int& lx, int& ly) {
    if (r < BX) { lx = r; ly = -1; }
    else if (r < 2 * BX) { lx = r - BX; ly = BY; }
    else if (r < 2 * BX + BY) { lx = -1; ly = r - 2 * BX; }
    else { lx = BX; ly = r - 2 * BX - BY; }
}

// Prefetch distance of the pair kernels' loads, in planes: each block keeps
// the loads of the next D planes in flight.  With the register rings one
// plane suffices for the momentum pairs (two push the FP64 pair 1 past 256
// registers, and gain nothing for pair 0 or in FP32); the FP64 scalar pairs
// gain 3% from two.
#ifndef DNSLAB_PAIR_DIST_MOM64
#define DNSLAB_PAIR_DIST_MOM64 1
#endif
#ifndef DNSLAB_PAIR_DIST_MOM64_P0
#define DNSLAB_PAIR_DIST_MOM64_P0 DNSLAB_PAIR_DIST_MOM64   // FP64 momentum pair 0 (fewer registers than pair 1)
#endif
#ifndef DNSLAB_PAIR_DIST_SCA64
#define DNSLAB_PAIR_DIST_SCA64 2   // FP64 scalar pairs: 2038 -> 1976 us on 1024x512x256 (201 / 235 registers)
#endif
#ifndef DNSLAB_PAIR_DIST_OTHER
#define DNSLAB_PAIR_DIST_OTHER 1
#endif
#ifndef DNSLAB_PAIR_DIST_MOM32_P0
#define DNSLAB_PAIR_DIST_MOM32_P0 DNSLAB_PAIR_DIST_OTHER   // FP32 momentum pair 0
#endif
// Waves per SIMD the FP32 pair kernels are compiled for (0: the compiler's
// choice).  Four keep them within 128 registers, two 512-thread blocks per
// CU (measured on 1024x512x256: momentum pairs 1747 -> 1621 us, scalar
// pairs 1318 -> 1243 us, against one block per CU at 133-151 registers).
#ifndef DNSLAB_PAIR_WAVES32
#define DNSLAB_PAIR_WAVES32 4
#endif
#ifndef DNSLAB_PAIR_WAVES32_MOM1
#define DNSLAB_PAIR_WAVES32_MOM1 DNSLAB_PAIR_WAVES32
#endif
// The FP32 scalar pair 1 needs 138 registers: held to 128 it spilled 19 per
// lane.  Unconstrained (one block per CU) it is 3% slower alone, but the
// FP32 step on 1024x512x256, where it runs beside the momentum pair 1 on the
// second stream, went from 8.10 to 8.24 Gcell-steps/s.
#ifndef DNSLAB_PAIR_WAVES32_SCA1
#define DNSLAB_PAIR_WAVES32_SCA1 0
#endif
#ifndef DNSLAB_PAIR_DIST_SCA32
#define DNSLAB_PAIR_DIST_SCA32 DNSLAB_PAIR_DIST_OTHER
#endif
template <typename T, bool MOM, int PAIR>
constexpr int pair_dist() {
    return sizeof(T) != 8 ? (MOM ? (PAIR == 0 ? DNSLAB_PAIR_DIST_MOM32_P0 : DNSLAB_PAIR_DIST_OTHER) : DNSLAB_PAIR_DIST_SCA32)
                          : (MOM ? (PAIR == 0 ? DNSLAB_PAIR_DIST_MOM64_P0 : DNSLAB_PAIR_DIST_MOM64) : DNSLAB_PAIR_DIST_SCA64);
}
template <typename T, bool MOM, int PAIR>
constexpr int pair_waves() {
    constexpr int w = sizeof(T) != 4 ? 0
                      : (PAIR == 1 ? (MOM ? DNSLAB_PAIR_WAVES32_MOM1 : DNSLAB_PAIR_WAVES32_SCA1) : DNSLAB_PAIR_WAVES32);
    return w > 0 ? w : 1;
}

// Register rings of the z-marching kernels (stage pairs, filter,
// correction).  A value belonging to z plane x of the march (x counted from
// the chunk's first iteration) sits in slot x % U of its ring, and the z loop
// is unrolled U times (pair_phases), so every slot index is a compile-time
// constant: values stay in the register they were loaded into.  Shifting a
// queue instead (q[i] = q[i+1]) costs a move per value and plane, and a move
// of a register whose load is still in flight makes the wave wait for that
// load, which defeats the prefetch.
template <int... Is, typename F>
__device__ __forceinline__ bool pair_phases(std::integer_sequence<int, Is...>, F&& f) {
    return (f(std::integral_constant<int, Is>{}) && ...);
}
// Loads and stores of the register-ring kernels as raw buffer accesses: the
// array's resource (base address) and the plane's byte offset are
// wave-uniform (scalar registers), the in-plane byte offset is the lane's
// (one vector register, fixed for the whole march), and the address is
// formed by the memory unit: no per-lane 64-bit address arithmetic, and
// nothing the compiler can hoist into one 64-bit pointer per array and lane.
// The resource does no range clipping (every offset is inside its array).
typedef unsigned u32x2_t __attribute__((__vector_size__(2 * sizeof(unsigned))));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_res(const void* p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, -1, 0x00020000);
}
template <typename T> struct BufIO;
template <> struct BufIO<double> {
    static __device__ __forceinline__ double ld(const void* p, unsigned v, unsigned s) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(buf_res(p), v, s, 0));
    }
    static __device__ __forceinline__ void st(void* p, unsigned v, unsigned s, double x) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, x), buf_res(p), v, s, 0);
    }
};
template <> struct BufIO<float> {
    static __device__ __forceinline__ float ld(const void* p, unsigned v, unsigned s) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(buf_res(p), v, s, 0));
    }
    static __device__ __forceinline__ void st(void* p, unsigned v, unsigned s, float x) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), buf_res(p), v, s, 0);
    }
};
template <> struct BufIO<uint8_t> {
    static __device__ __forceinline__ uint8_t ld(const void* p, unsigned v, unsigned s) {
        return __builtin_amdgcn_raw_buffer_load_b8(buf_res(p), v, s, 0);
    }
};
// element at byte offset voff of the plane at byte offset soff
template <typename T>
__device__ __forceinline__ T bld(const T* p, unsigned voff, unsigned soff) { return BufIO<T>::ld(p, voff, soff); }
template <typename T>
__device__ __forceinline__ void bst(T* p, unsigned voff, unsigned soff, T x) { BufIO<T>::st(p, voff, soff, x); }
// A per-lane value the compiler must take as redefined at this point.  The
// register-ring kernels (stage pairs, filter, correction) pass their LDS
// indices through it once per plane: otherwise
// the address of every LDS access of the unrolled march (a different
// constant offset per plane of the buffer cycle) is hoisted out of the loop
// and held in a register of its own for the whole kernel.
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}
// Offsets of planes K + s (s = 0, 1, 1 + D, 2 + D, wrapped periodically),
// advanced by one plane per iteration without a division.
template <int D>
struct PlaneOffsets {
    unsigned p0, p1, pd1, pd2;
    unsigned nxy, ntot;
    __device__ __forceinline__ PlaneOffsets(int K, int nz, unsigned nxy_) : nxy(nxy_), ntot((unsigned)nz * nxy_) {
        p0 = (unsigned)wrap(K, nz) * nxy;
        p1 = (unsigned)wrap(K + 1, nz) * nxy;
        pd1 = (unsigned)wrap(K + 1 + D, nz) * nxy;
        pd2 = (unsigned)wrap(K + 2 + D, nz) * nxy;
    }
    __device__ __forceinline__ static unsigned step(unsigned p, unsigned nxy, unsigned ntot) {
        p += nxy;
        return p == ntot ? 0u : p;
    }
    __device__ __forceinline__ void advance() {
        p0 = step(p0, nxy, ntot);
        p1 = step(p1, nxy, ntot);
        pd1 = step(pd1, nxy, ntot);
        pd2 = step(pd2, nxy, ntot);
    }
};

template <typename T, int PAIR, int D, int BY>
__device__ __forceinline__ void mom_pair_body(const MomPairArgs<T>& a, const BlockIdx3& bi) {
    constexpr int BX = 64;
    constexpr int U = (4 + D) & ~1;                   // ring slots: even (LDS buffer parity), >= 3 + D
    constexpr int WV = BX + 4, TV = WV * (BY + 4);    // V tile: radius 2, per component
    constexpr int WW = BX + 2, TW = WW * (BY + 2);    // W tile: radius 1, per component
    constexpr int NRING = 2 * (BX + BY);
    constexpr int HM = (4 * (BX + 2) + 4 * BY + BX * BY - 1) / (BX * BY);   // halo cells per thread
    constexpr unsigned E = sizeof(T);
    const Grid& g = a.g;
    const Col col = column(g, a.kc, bi);
    const int k0 = col.k0, k1 = col.k1;
    const T dt = T(a.dtp ? *a.dtp : a.dt);
    const MomCoef<T> cf = mom_coef<T>(g, a.nu, a.body);
    extern __shared__ unsigned char smem_raw[];
    T* const Vb = reinterpret_cast<T*>(smem_raw);    // [2 planes][3 components][TV]
    T* const Wb = Vb + 6 * TV;                       // [2 planes][3 components][TW]
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + BX * ty;
    const int i0 = col.i - tx, j0 = col.j - ty;
    const unsigned cell = col.row + col.i;
    const unsigned cb = cell * E;
    const int cV0 = (ty + 2) * WV + tx + 2, cW0 = (ty + 1) * WW + tx + 1;
    const PairHalo<HM> hm = pair_halo<HM>(i0, j0, g, BX, BY, tid, BX * BY);
    unsigned hb[HM];
#pragma unroll
    for (int h = 0; h < HM; ++h) hb[h] = hm.src[h] * E;
    // this thread's ring cell, if any
    const bool ring = tid < NRING;
    int rlx = 0, rly = 0;
    if (ring) ring_cell(tid, BX, BY, rlx, rly);
    const unsigned rcell = (unsigned)wrap1(j0 + rly, g.ny) * g.nx + (unsigned)wrap1(i0 + rlx, g.nx);
    const unsigned rcb = rcell * E;
    const int rV0 = (rly + 2) * WV + rlx + 2, rW0 = (rly + 1) * WW + rlx + 1;

    // Rings, by plane of the march:
    //   vq: stage input of this thread's cell (planes K .. K+2+D live in iteration K)
    //   hq: V halo (planes K+2 .. K+2+D, staged into LDS at K+2)
    //   fq: flags of the cell; rfq: flags of the ring cell
    //   unq, runq, acq (pair 1): u^n of cell and ring cell, acc after stage 2
    //   wz: first-stage value of the cell; ac: its running accumulator
    //   rv: the ring cell's stage input (its z- neighbour one plane later)
    T vq[U][3], hq[U][3][HM], unq[U][3], runq[U][3], acq[U][3], wz[U][3], ac[U][3], rv[U][3];
    uint8_t fq[U], rfq[U];
#pragma unroll
    for (int s = 0; s < U; ++s) {
        fq[s] = 0;
        rfq[s] = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            vq[s][c] = T(0); unq[s][c] = T(0); runq[s][c] = T(0); acq[s][c] = T(0);
            wz[s][c] = T(0); ac[s][c] = T(0); rv[s][c] = T(0);
#pragma unroll
            for (int h = 0; h < HM; ++h) hq[s][c][h] = T(0);
        }
    }
    PlaneOffsets<D> po(k0 - 2, g.nz, (unsigned)g.nxy);
    {
        // iteration 0 is plane K = k0 - 2
        const int K = k0 - 2;
#pragma unroll
        for (int i = 0; i < 2 + D; ++i) {
            const unsigned pi = (unsigned)wrap(K + i, g.nz) * g.nxy;
#pragma unroll
            for (int c = 0; c < 3; ++c) vq[i][c] = bld(a.vin[c], cb, pi * E);
        }
#pragma unroll
        for (int i = 1; i < 1 + D; ++i) fq[i] = a.flags[(unsigned)wrap(K + i, g.nz) * g.nxy + cell];
#pragma unroll
        for (int i = 1; i < 1 + D; ++i) {
            const unsigned pi = (unsigned)wrap(K + i, g.nz) * g.nxy;
            if (ring) rfq[i] = a.flags[pi + rcell];
            if (PAIR == 1) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    unq[i][c] = bld(a.un[c], cb, pi * E);
                    if (ring) runq[i][c] = bld(a.un[c], rcb, pi * E);
                    if (K + i >= k0 && K + i < k1) acq[i][c] = bld(a.accin[c], cb, pi * E);
                }
            }
        }
        if (ring) {
#pragma unroll
            for (int c = 0; c < 3; ++c) rv[0][c] = bld(a.vin[c], rcb, po.p0 * E);
        }
        // V tile of plane k0 - 1 (buffer 1)
        T* Vp = Vb + 3 * TV;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Vp[c * TV + cV0] = vq[1][c];
#pragma unroll
            for (int h = 0; h < HM; ++h)
                if (h < hm.n) Vp[c * TV + hm.dst[h]] = bld(a.vin[c], hb[h], po.p1 * E);
        }
        // halos of planes k0 .. k0 + D - 1
#pragma unroll
        for (int i = 2; i < 2 + D; ++i) {
            const unsigned pi = (unsigned)wrap(K + i, g.nz) * g.nxy;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int h = 0; h < HM; ++h) hq[i][c][h] = h < hm.n ? bld(a.vin[c], hb[h], pi * E) : T(0);
        }
    }

    const int nit = k1 - k0 + 2;
    int r = 0;   // iteration: K = k0 - 2 + r
    auto iter = [&](auto phase) __attribute__((always_inline)) -> bool {
        constexpr int P = decltype(phase)::value;
        constexpr int S0 = P % U, S1 = (P + 1) % U, S2 = (P + 2) % U, SM = (P + U - 1) % U;
        constexpr int SD1 = (P + 1 + D) % U, SD2 = (P + 2 + D) % U;
        if (r >= nit) return false;
        const int K = k0 - 2 + r;
        const int cV = opaque(cV0), cW = opaque(cW0), rV = opaque(rV0), rW = opaque(rW0);
        int hd[HM];
#pragma unroll
        for (int h = 0; h < HM; ++h) hd[h] = opaque(hm.dst[h]);
        // 1. stage input of plane K + 2 into V (buffer parity of K + 2)
        T* const Vq = Vb + (P & 1) * 3 * TV;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Vq[c * TV + cV] = vq[S2][c];
#pragma unroll
            for (int h = 0; h < HM; ++h)
                if (h < hm.n) Vq[c * TV + hd[h]] = hq[S2][c][h];
        }
        // 2. loads D planes ahead: v and halo of plane K + 2 + D, the rest of
        // plane K + 1 + D.  Past the chunk's last plane the loads still run,
        // from plane K (valid memory, never used): a slot written on every
        // path leaves its value of U planes earlier dead, and no branch or
        // select on the loaded values is needed.
        {
            const bool more = K + D < k1;
            const unsigned sv = (more ? po.pd2 : po.p0) * E, sr = (more ? po.pd1 : po.p0) * E;
            const unsigned fr = more ? po.pd1 : po.p0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                vq[SD2][c] = bld(a.vin[c], cb, sv);
#pragma unroll
                for (int h = 0; h < HM; ++h) {
                    hq[SD2][c][h] = T(0);
                    if (h < hm.n) hq[SD2][c][h] = bld(a.vin[c], hb[h], sv);
                }
            }
            fq[SD1] = bld(a.flags, cell, fr);
            rfq[SD1] = 0;
            if (ring) rfq[SD1] = bld(a.flags, rcell, fr);
            if (PAIR == 1) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    unq[SD1][c] = bld(a.un[c], cb, sr);
                    runq[SD1][c] = T(0);
                    if (ring) runq[SD1][c] = bld(a.un[c], rcb, sr);
                    acq[SD1][c] = bld(a.accin[c], cb, sr);
                }
            }
        }
        __syncthreads();
        // 3. first stage at plane K + 1: w on the tile and the ring
        const T* const Vp = Vb + ((P + 1) & 1) * 3 * TV;
        T* const Wp = Wb + ((P + 1) & 1) * 3 * TW;
        {
            T xm[3], xp[3], ym[3], yp[3], kv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                xm[c] = Vp[c * TV + cV - 1];
                xp[c] = Vp[c * TV + cV + 1];
                ym[c] = Vp[c * TV + cV - WV];
                yp[c] = Vp[c * TV + cV + WV];
            }
            mom_rhs_cell<T>(cf, vq[S1], xm, xp, ym, yp, vq[S0], vq[S2], fq[S1], a.frc, po.p1 + cell, kv);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (PAIR == 0) {
                    ac[S1][c] = vq[S1][c] + (dt / T(6)) * kv[c];
                    wz[S1][c] = vq[S1][c] + (dt / T(2)) * kv[c];
                } else {
                    ac[S1][c] = acq[S1][c] + (dt / T(3)) * kv[c];
                    wz[S1][c] = unq[S1][c] + dt * kv[c];
                }
                Wp[c * TW + cW] = wz[S1][c];
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) rv[S1][c] = T(0);
        if (ring) {
            T c0[3], xm[3], xp[3], ym[3], yp[3], zp[3], kv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                c0[c] = Vp[c * TV + rV];
                xm[c] = Vp[c * TV + rV - 1];
                xp[c] = Vp[c * TV + rV + 1];
                ym[c] = Vp[c * TV + rV - WV];
                yp[c] = Vp[c * TV + rV + WV];
                zp[c] = Vq[c * TV + rV];
            }
            mom_rhs_cell<T>(cf, c0, xm, xp, ym, yp, rv[S0], zp, rfq[S1], a.frc, po.p1 + rcell, kv);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Wp[c * TW + rW] = PAIR == 0 ? c0[c] + (dt / T(2)) * kv[c] : runq[S1][c] + dt * kv[c];
                rv[S1][c] = c0[c];
            }
        }
        __syncthreads();
        // 4. second stage at plane K
        if (r >= 2) {
            const T* const Wk = Wb + (P & 1) * 3 * TW;
            T xm[3], xp[3], ym[3], yp[3], kv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                xm[c] = Wk[c * TW + cW - 1];
                xp[c] = Wk[c * TW + cW + 1];
                ym[c] = Wk[c * TW + cW - WW];
                yp[c] = Wk[c * TW + cW + WW];
            }
            mom_rhs_cell<T>(cf, wz[S0], xm, xp, ym, yp, wz[SM], wz[S1], fq[S0], a.frc, po.p0 + cell, kv);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (PAIR == 0) {
                    bst(a.acc[c], cb, po.p0 * E, ac[S0][c] + (dt / T(3)) * kv[c]);
                    bst(a.out[c], cb, po.p0 * E, vq[S0][c] + (dt / T(2)) * kv[c]);
                } else {
                    bst(a.out[c], cb, po.p0 * E, ac[S0][c] + (dt / T(6)) * kv[c]);
                }
            }
        }
        po.advance();
        ++r;
        return true;
    };
    while (pair_phases(std::make_integer_sequence<int, U>{}, iter)) {
    }
}

// ---------------------------------------------------------------------------
// Scalar RK4 stage.  G = beta [ -sum_a D_a(u_a c) + alpha div(beta grad c)
//                              + S (c_set - c)/tau_f ],
// the masked diffusion conducting only across fluid-fluid faces.
// ---------------------------------------------------------------------------
template <typename T>
struct ScaCoef {
    T h2x, h2y, h2z, ix2, iy2, iz2, alpha;
};
template <typename T>
__device__ __forceinline__ ScaCoef<T> sca_coef(const Grid& g, double alpha) {
    ScaCoef<T> c;
    c.h2x = T(g.inv2d[0]); c.h2y = T(g.inv2d[1]); c.h2z = T(g.inv2d[2]);
    c.ix2 = T(g.invd2[0]); c.iy2 = T(g.invd2[1]); c.iz2 = T(g.invd2[2]);
    c.alpha = T(alpha);
    return c;
}

// G(c) at one cell from c at the cell and its six face neighbours, the
// velocity component normal to each face pair at those neighbours, and the
// flags (every scalar kernel evaluates G through this one function).
template <typename T>
__device__ __forceinline__ T sca_rhs_cell(const ScaCoef<T>& cf, T c0, T cxm, T cxp, T cym, T cyp, T cm, T cp,
                                          T uxm, T uxp, T vym, T vyp, T wm, T wp, uint8_t f0, uint8_t fxm,
                                          uint8_t fxp, uint8_t fym, uint8_t fyp, uint8_t fm, uint8_t fp,
                                          const Forcing& frc, unsigned idx) {
    T G = T(0);
    if (f0 & F_FLUID) {
        const T conv = (uxp * cxp - uxm * cxm) * cf.h2x + (vyp * cyp - vym * cym) * cf.h2y + (wp * cp - wm * cm) * cf.h2z;
        const T lx = ((fxp & F_FLUID) ? cxp - c0 : T(0)) - ((fxm & F_FLUID) ? c0 - cxm : T(0));
        const T ly = ((fyp & F_FLUID) ? cyp - c0 : T(0)) - ((fym & F_FLUID) ? c0 - cym : T(0));
        const T lz = ((fp & F_FLUID) ? cp - c0 : T(0)) - ((fm & F_FLUID) ? c0 - cm : T(0));
        G = -conv + cf.alpha * (lx * cf.ix2 + ly * cf.iy2 + lz * cf.iz2);
        if (f0 & F_FORCED) {
            const int e = forced_entry(frc, (long long)idx);
            G += T(frc.S[e]) * T(frc.inv_tau) * (T(frc.cset[e]) - c0);
        }
    }
    return G;
}

template <typename T, int MODE>
__device__ __forceinline__ void sca_stage_body(const ScaArgs<T>& a, const BlockIdx3& bi) {
    const Grid& g = a.g;
    const Col col = column(g, a.kc, bi);
    const int k0 = col.k0, k1 = col.k1;
    const unsigned nxy = (unsigned)g.nxy;
    const T dt = (MODE == ST_RHS) ? T(0) : T(a.dtp ? *a.dtp : a.dt);
    const ScaCoef<T> cf = sca_coef<T>(g, a.alpha);
    const T* __restrict__ cs = a.cs;
    const T* __restrict__ ux = a.u[0];
    const T* __restrict__ uy = a.u[1];
    const T* __restrict__ uz = a.u[2];
    Partial part = {0, 0, 0, 0, 0, 0};

    if (col.active) {
        T cm, c0, cp, wm, w0, wp;
        uint8_t fm, f0, fp;
        {
            const int km = k0 == 0 ? g.nz - 1 : k0 - 1;
            const unsigned im_ = (unsigned)km * nxy + col.row + col.i;
            const unsigned i0_ = (unsigned)k0 * nxy + col.row + col.i;
            cm = cs[im_]; c0 = cs[i0_];
            wm = uz[im_]; w0 = uz[i0_];
            fm = a.flags[im_]; f0 = a.flags[i0_];
        }
        for (int k = k0; k < k1; ++k) {
            const int kp = k + 1 == g.nz ? 0 : k + 1;
            const unsigned base = (unsigned)k * nxy;
            const unsigned idx = base + col.row + col.i;
            const unsigned ipz = (unsigned)kp * nxy + col.row + col.i;
            cp = cs[ipz]; wp = uz[ipz]; fp = a.flags[ipz];
            const unsigned ixm = base + col.row + col.im, ixp = base + col.row + col.ip;
            const unsigned iym = base + col.rowm + col.i, iyp = base + col.rowp + col.i;
            const T cxm = cs[ixm], cxp = cs[ixp], cym = cs[iym], cyp = cs[iyp];
            const T uxm = ux[ixm], uxp = ux[ixp], vym = uy[iym], vyp = uy[iyp];
            const uint8_t fxm = a.flags[ixm], fxp = a.flags[ixp], fym = a.flags[iym], fyp = a.flags[iyp];

            const T G = sca_rhs_cell<T>(cf, c0, cxm, cxp, cym, cyp, cm, cp, uxm, uxp, vym, vyp, wm, wp, f0, fxm, fxp,
                                        fym, fyp, fm, fp, a.frc, idx);
            if (MODE == ST_FIRST) {
                a.acc[idx] = c0 + (dt / T(6)) * G;
                a.out[idx] = c0 + (dt / T(2)) * G;
                if (a.part.p) {
                    const double dv = ((double)uxp - (double)uxm) * g.inv2d[0] + ((double)vyp - (double)vym) * g.inv2d[1] +
                                      ((double)wp - (double)wm) * g.inv2d[2];
                    part.div2 += dv * dv;
                }
            } else if (MODE == ST_HALF || MODE == ST_FULL) {
                const T cn = a.cn[idx];
                a.acc[idx] = a.acc[idx] + (dt / T(3)) * G;
                a.out[idx] = cn + (MODE == ST_HALF ? dt / T(2) : dt) * G;
            } else if (MODE == ST_LAST) {
                const T cnew = (f0 & F_FLUID) ? a.acc[idx] + (dt / T(6)) * G : T(0);
                a.out[idx] = cnew;
                if (a.part.p) {
                    const double b = (f0 & F_FLUID) ? 1.0 : 0.0;
                    part.mass += b * (double)cnew;
                    if (f0 & F_ROOM) { part.room_num += b * (double)cnew; part.room_den += b; }
                }
            } else {
                a.out[idx] = G;
            }
            cm = c0; c0 = cp; wm = w0; w0 = wp; fm = f0; f0 = fp;
        }
    }
    if (MODE == ST_FIRST && a.part.p) block_reduce_partial<PM_DIV>(part, a.part, (int)bi.hw);
    if (MODE == ST_LAST && a.part.p) block_reduce_partial<PM_SCA>(part, a.part, (int)bi.hw);
}

// ---------------------------------------------------------------------------
// Two scalar RK4 stages in one pass (ScaPairArgs), with the pipeline of
// mom_pair_body.  The first stage at plane K+1 needs c with a radius-2 halo,
// u and v at x and y neighbours and the flags with a radius-2 halo, so c, u,
// v and the flags of planes K+1 and K+2 are staged in LDS; w is only needed at
// z neighbours (the threads' own z windows, and the ring cells' own).  The
// second stage at plane K needs u, v and the flags at the same neighbours the
// first stage read one plane earlier: each thread keeps them from there.
// ---------------------------------------------------------------------------
template <typename T, int PAIR, int D, int BY>
__device__ __forceinline__ void sca_pair_body(const ScaPairArgs<T>& a, const BlockIdx3& bi) {
    constexpr int BX = 64;
    constexpr int U = (5 + D) & ~1;                   // ring slots: even (LDS buffer parity), >= 4 + D
    constexpr int WV = BX + 4, TV = WV * (BY + 4);
    constexpr int WW = BX + 2, TW = WW * (BY + 2);
    constexpr int NRING = 2 * (BX + BY);
    constexpr int HM = (4 * (BX + 2) + 4 * BY + BX * BY - 1) / (BX * BY);
    constexpr unsigned E = sizeof(T);
    const Grid& g = a.g;
    const Col col = column(g, a.kc, bi);
    const int k0 = col.k0, k1 = col.k1;
    const T dt = T(a.dtp ? *a.dtp : a.dt);
    const ScaCoef<T> cf = sca_coef<T>(g, a.alpha);
    extern __shared__ unsigned char smem_raw[];
    T* const Cs = reinterpret_cast<T*>(smem_raw);   // c, 2 planes
    T* const Us = Cs + 2 * TV;                        // u, 2 planes
    T* const Vs = Us + 2 * TV;                        // v, 2 planes
    T* const Ws = Vs + 2 * TV;                        // first-stage value c1, 2 planes (radius 1)
    uint8_t* const Fs = reinterpret_cast<uint8_t*>(Ws + 2 * TW);   // flags, 2 planes
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + BX * ty;
    const int i0 = col.i - tx, j0 = col.j - ty;
    const unsigned cell = col.row + col.i;
    const unsigned cb = cell * E;
    const int cV0 = (ty + 2) * WV + tx + 2, cW0 = (ty + 1) * WW + tx + 1;
    const PairHalo<HM> hm = pair_halo<HM>(i0, j0, g, BX, BY, tid, BX * BY);
    unsigned hb[HM];
#pragma unroll
    for (int h = 0; h < HM; ++h) hb[h] = hm.src[h] * E;
    const bool ring = tid < NRING;
    int rlx = 0, rly = 0;
    if (ring) ring_cell(tid, BX, BY, rlx, rly);
    const unsigned rcell = (unsigned)wrap1(j0 + rly, g.ny) * g.nx + (unsigned)wrap1(i0 + rlx, g.nx);
    const unsigned rcb = rcell * E;
    const int rV0 = (rly + 2) * WV + rlx + 2, rW0 = (rly + 1) * WW + rlx + 1;
    Partial part = {0, 0, 0, 0, 0, 0};

    // Rings, by plane of the march (iteration K):
    //   cq: c_in of the cell (planes K .. K+2+D); wq, fq: w and flags of the
    //   cell (planes K-1 .. K+2+D); uq, vq and the halo rings: planes
    //   K+2 .. K+2+D, staged into LDS at K+2; rwq: the ring cell's w;
    //   cnq, rcnq, acq (pair 1): c^n of cell and ring cell, acc after stage 2;
    //   c1: first-stage value of the cell; ac: its accumulator;
    //   sx, sf: u, v and flags at the cell's x/y neighbours, read by the first
    //   stage of plane K+1 and used again by the second stage there;
    //   rc, rf: the ring cell's c and flags.
    T cq[U], wq[U], uq[U], vq[U], hc[U][HM], hu[U][HM], hv[U][HM], rwq[U];
    T cnq[U], rcnq[U], acq[U], c1[U], ac[U], sx[U][4], rc[U];
    uint8_t fq[U], hf[U][HM], sf[U][4], rf[U];
#pragma unroll
    for (int s = 0; s < U; ++s) {
        cq[s] = T(0); wq[s] = T(0); uq[s] = T(0); vq[s] = T(0); rwq[s] = T(0);
        cnq[s] = T(0); rcnq[s] = T(0); acq[s] = T(0); c1[s] = T(0); ac[s] = T(0); rc[s] = T(0);
        fq[s] = 0; rf[s] = 0;
#pragma unroll
        for (int h = 0; h < HM; ++h) { hc[s][h] = T(0); hu[s][h] = T(0); hv[s][h] = T(0); hf[s][h] = 0; }
#pragma unroll
        for (int q = 0; q < 4; ++q) { sx[s][q] = T(0); sf[s][q] = 0; }
    }
    const T* __restrict__ ux = a.u[0];
    const T* __restrict__ uy = a.u[1];
    const T* __restrict__ uz = a.u[2];
    PlaneOffsets<D> po(k0 - 2, g.nz, (unsigned)g.nxy);
    {
        const int K = k0 - 2;
        auto pl = [&](int k) -> unsigned { return (unsigned)wrap(k, g.nz) * g.nxy; };
#pragma unroll
        for (int i = 0; i < 2 + D; ++i) {
            const unsigned pi = pl(K + i);
            cq[i] = bld(a.cin, cb, pi * E);
            wq[i] = bld(uz, cb, pi * E);
            fq[i] = a.flags[pi + cell];
            if (ring) rwq[i] = bld(uz, rcb, pi * E);
        }
#pragma unroll
        for (int i = 2; i < 2 + D; ++i) {
            const unsigned pi = pl(K + i);
            uq[i] = bld(ux, cb, pi * E);
            vq[i] = bld(uy, cb, pi * E);
#pragma unroll
            for (int h = 0; h < HM; ++h) {
                const bool on = h < hm.n;
                hc[i][h] = on ? bld(a.cin, hb[h], pi * E) : T(0);
                hu[i][h] = on ? bld(ux, hb[h], pi * E) : T(0);
                hv[i][h] = on ? bld(uy, hb[h], pi * E) : T(0);
                hf[i][h] = on ? a.flags[pi + hm.src[h]] : 0;
            }
        }
        if (ring) {
            rc[0] = bld(a.cin, rcb, po.p0 * E);
            rf[0] = a.flags[po.p0 + rcell];
        }
        if (PAIR == 1) {
#pragma unroll
            for (int i = 1; i < 1 + D; ++i) {
                const unsigned pi = pl(K + i);
                cnq[i] = bld(a.cn, cb, pi * E);
                if (ring) rcnq[i] = bld(a.cn, rcb, pi * E);
                if (K + i >= k0 && K + i < k1) acq[i] = bld(a.accin, cb, pi * E);
            }
        }
        // LDS planes of k0 - 1 (buffer 1)
        const unsigned pb = po.p1;
        Cs[TV + cV0] = cq[1];
        Us[TV + cV0] = bld(ux, cb, pb * E);
        Vs[TV + cV0] = bld(uy, cb, pb * E);
        Fs[TV + cV0] = fq[1];
#pragma unroll
        for (int h = 0; h < HM; ++h)
            if (h < hm.n) {
                Cs[TV + hm.dst[h]] = bld(a.cin, hb[h], pb * E);
                Us[TV + hm.dst[h]] = bld(ux, hb[h], pb * E);
                Vs[TV + hm.dst[h]] = bld(uy, hb[h], pb * E);
                Fs[TV + hm.dst[h]] = a.flags[pb + hm.src[h]];
            }
    }

    const int nit = k1 - k0 + 2;
    int r = 0;   // iteration: K = k0 - 2 + r
    auto iter = [&](auto phase) __attribute__((always_inline)) -> bool {
        constexpr int P = decltype(phase)::value;
        constexpr int S0 = P % U, S1 = (P + 1) % U, S2 = (P + 2) % U, SM = (P + U - 1) % U;
        constexpr int SD1 = (P + 1 + D) % U, SD2 = (P + 2 + D) % U;
        constexpr int bq = P & 1, bp = (P + 1) & 1;   // LDS buffers of planes K + 2 and K + 1
        if (r >= nit) return false;
        const int K = k0 - 2 + r;
        const int cV = opaque(cV0), cW = opaque(cW0), rV = opaque(rV0), rW = opaque(rW0);
        int hd[HM];
#pragma unroll
        for (int h = 0; h < HM; ++h) hd[h] = opaque(hm.dst[h]);
        // 1. plane K + 2 into LDS
        Cs[bq * TV + cV] = cq[S2];
        Us[bq * TV + cV] = uq[S2];
        Vs[bq * TV + cV] = vq[S2];
        Fs[bq * TV + cV] = fq[S2];
#pragma unroll
        for (int h = 0; h < HM; ++h)
            if (h < hm.n) {
                Cs[bq * TV + hd[h]] = hc[S2][h];
                Us[bq * TV + hd[h]] = hu[S2][h];
                Vs[bq * TV + hd[h]] = hv[S2][h];
                Fs[bq * TV + hd[h]] = hf[S2][h];
            }
        // 2. loads D planes ahead (past the chunk's end from plane K, as in
        // mom_pair_body)
        {
            const bool more = K + D < k1;
            const unsigned pv = more ? po.pd2 : po.p0, pr = more ? po.pd1 : po.p0;
            cq[SD2] = bld(a.cin, cb, pv * E);
            wq[SD2] = bld(uz, cb, pv * E);
            fq[SD2] = bld(a.flags, cell, pv);
            uq[SD2] = bld(ux, cb, pv * E);
            vq[SD2] = bld(uy, cb, pv * E);
#pragma unroll
            for (int h = 0; h < HM; ++h) {
                hc[SD2][h] = T(0); hu[SD2][h] = T(0); hv[SD2][h] = T(0); hf[SD2][h] = 0;
                if (h < hm.n) {
                    hc[SD2][h] = bld(a.cin, hb[h], pv * E);
                    hu[SD2][h] = bld(ux, hb[h], pv * E);
                    hv[SD2][h] = bld(uy, hb[h], pv * E);
                    hf[SD2][h] = bld(a.flags, hm.src[h], pv);
                }
            }
            rwq[SD2] = T(0);
            if (ring) rwq[SD2] = bld(uz, rcb, pv * E);
            if (PAIR == 1) {
                cnq[SD1] = bld(a.cn, cb, pr * E);
                rcnq[SD1] = T(0);
                if (ring) rcnq[SD1] = bld(a.cn, rcb, pr * E);
                acq[SD1] = bld(a.accin, cb, pr * E);
            }
        }
        __syncthreads();
        // 3. first stage at plane K + 1 on the tile and the ring
        T* const Wp = Ws + bp * TW;
        {
            const T* C = Cs + bp * TV;
            const T* Uu = Us + bp * TV;
            const T* V = Vs + bp * TV;
            const uint8_t* F = Fs + bp * TV;
            sx[S1][0] = Uu[cV - 1]; sx[S1][1] = Uu[cV + 1]; sx[S1][2] = V[cV - WV]; sx[S1][3] = V[cV + WV];
            sf[S1][0] = F[cV - 1]; sf[S1][1] = F[cV + 1]; sf[S1][2] = F[cV - WV]; sf[S1][3] = F[cV + WV];
            const T G = sca_rhs_cell<T>(cf, cq[S1], C[cV - 1], C[cV + 1], C[cV - WV], C[cV + WV], cq[S0], cq[S2],
                                        sx[S1][0], sx[S1][1], sx[S1][2], sx[S1][3], wq[S0], wq[S2], fq[S1],
                                        sf[S1][0], sf[S1][1], sf[S1][2], sf[S1][3], fq[S0], fq[S2], a.frc,
                                        po.p1 + cell);
            if (PAIR == 0) {
                ac[S1] = cq[S1] + (dt / T(6)) * G;
                c1[S1] = cq[S1] + (dt / T(2)) * G;
            } else {
                ac[S1] = acq[S1] + (dt / T(3)) * G;
                c1[S1] = cnq[S1] + dt * G;
            }
            Wp[cW] = c1[S1];
            rc[S1] = T(0);
            rf[S1] = 0;
            if (ring) {
                const T* Cq = Cs + bq * TV;
                const uint8_t* Fq = Fs + bq * TV;
                const T rc0 = C[rV];
                const uint8_t rf0 = F[rV];
                const T Gr = sca_rhs_cell<T>(cf, rc0, C[rV - 1], C[rV + 1], C[rV - WV], C[rV + WV], rc[S0], Cq[rV],
                                             Uu[rV - 1], Uu[rV + 1], V[rV - WV], V[rV + WV], rwq[S0], rwq[S2], rf0,
                                             F[rV - 1], F[rV + 1], F[rV - WV], F[rV + WV], rf[S0], Fq[rV], a.frc,
                                             po.p1 + rcell);
                Wp[rW] = PAIR == 0 ? rc0 + (dt / T(2)) * Gr : rcnq[S1] + dt * Gr;
                rc[S1] = rc0;
                rf[S1] = rf0;
            }
        }
        __syncthreads();
        // 4. second stage at plane K on the tile
        if (r >= 2) {
            const T* Wk = Ws + bq * TW;
            const T G = sca_rhs_cell<T>(cf, c1[S0], Wk[cW - 1], Wk[cW + 1], Wk[cW - WW], Wk[cW + WW], c1[SM], c1[S1],
                                        sx[S0][0], sx[S0][1], sx[S0][2], sx[S0][3], wq[SM], wq[S1], fq[S0],
                                        sf[S0][0], sf[S0][1], sf[S0][2], sf[S0][3], fq[SM], fq[S1], a.frc,
                                        po.p0 + cell);
            if (PAIR == 0) {
                bst(a.acc, cb, po.p0 * E, ac[S0] + (dt / T(3)) * G);
                bst(a.out, cb, po.p0 * E, cq[S0] + (dt / T(2)) * G);
                if (a.part.p) {
                    const double dv = ((double)sx[S0][1] - (double)sx[S0][0]) * g.inv2d[0] +
                                      ((double)sx[S0][3] - (double)sx[S0][2]) * g.inv2d[1] +
                                      ((double)wq[S1] - (double)wq[SM]) * g.inv2d[2];
                    part.div2 += dv * dv;
                }
            } else {
                const T cnew = (fq[S0] & F_FLUID) ? ac[S0] + (dt / T(6)) * G : T(0);
                bst(a.out, cb, po.p0 * E, cnew);
                if (a.part.p) {
                    const double b = (fq[S0] & F_FLUID) ? 1.0 : 0.0;
                    part.mass += b * (double)cnew;
                    if (fq[S0] & F_ROOM) { part.room_num += b * (double)cnew; part.room_den += b; }
                }
            }
        }
        po.advance();
        ++r;
        return true;
    };
    while (pair_phases(std::make_integer_sequence<int, U>{}, iter)) {
    }
    if (PAIR == 0 && a.part.p) block_reduce_partial<PM_DIV>(part, a.part, (int)bi.hw);
    if (PAIR == 1 && a.part.p) block_reduce_partial<PM_SCA>(part, a.part, (int)bi.hw);
}

// ---------------------------------------------------------------------------
// Sixth-order filter of Section 2.1 with the undivided seven-point difference:
// out = beta (f + pi^-6 sum_a delta6_a f).
// ---------------------------------------------------------------------------
template <typename T, int NF>
__device__ __forceinline__ void filter_body(const FiltArgs<T>& a, const BlockIdx3& bi) {
    const Grid& g = a.g;
    const Col col = column(g, a.kc, bi);
    const int k0 = col.k0, k1 = col.k1;
    const unsigned nxy = (unsigned)g.nxy;
    const T c6 = T(INV_PI6);
    Partial part = {0, 0, 0, 0, 0, 0};
    if (col.active) {
        int ix[7], jy[7];
#pragma unroll
        for (int m = -3; m <= 3; ++m) {
            ix[m + 3] = wrap(col.i + m, g.nx);
            jy[m + 3] = wrap(col.j + m, g.ny) * g.nx;
        }
        // win[f][m] holds plane k + (m - 3) dir; the z difference only uses the
        // symmetric pairs (m, 6 - m), so either direction gives the same sums.
        const int dir = col.dir;
        const int ks = dir > 0 ? k0 : k1 - 1;
        T win[NF][7];
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                const int kk = wrap(ks + (m - 3) * dir, g.nz);
                win[f][m] = a.in[f][(unsigned)kk * nxy + col.row + col.i];
            }
        for (int k = ks, left = k1 - k0; left > 0; --left, k += dir) {
            const unsigned base = (unsigned)k * nxy;
            const unsigned idx = base + col.row + col.i;
            const int kk = wrap(k + 3 * dir, g.nz);
            const uint8_t fl = a.flags[idx];
            T res[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const T* __restrict__ src = a.in[f];
                win[f][6] = src[(unsigned)kk * nxy + col.row + col.i];
                const T f0 = win[f][3];
                const T* rowp = src + base + col.row;
                const T dx6 = (rowp[ix[0]] + rowp[ix[6]]) - T(6) * (rowp[ix[1]] + rowp[ix[5]]) +
                              T(15) * (rowp[ix[2]] + rowp[ix[4]]) - T(20) * f0;
                const T* colp = src + base + col.i;
                const T dy6 = (colp[jy[0]] + colp[jy[6]]) - T(6) * (colp[jy[1]] + colp[jy[5]]) +
                              T(15) * (colp[jy[2]] + colp[jy[4]]) - T(20) * f0;
                const T dz6 = (win[f][0] + win[f][6]) - T(6) * (win[f][1] + win[f][5]) +
                              T(15) * (win[f][2] + win[f][4]) - T(20) * f0;
                res[f] = (fl & F_FLUID) ? f0 + c6 * (dx6 + dy6 + dz6) : T(0);
                a.out[f][idx] = res[f];
#pragma unroll
                for (int m = 0; m < 6; ++m) win[f][m] = win[f][m + 1];
            }
            if (a.part.p) {
                const double b = (fl & F_FLUID) ? 1.0 : 0.0;
                if (NF == 3) {
                    const double u = (double)res[0], v = (double)res[1], w = (double)res[2];
                    part.ke += b * (u * u + v * v + w * w);
                    part.rate = fmax(part.rate, courant_rate(u, v, w, g));
                } else {
                    const double c = (double)res[0];
                    part.mass += b * c;
                    if (fl & F_ROOM) { part.room_num += b * c; part.room_den += b; }
                }
            }
        }
    }
    if (a.part.p) block_reduce_partial<NF == 3 ? PM_VEL : PM_SCA>(part, a.part, (int)bi.hw);
}

// The same filter with the x and y neighbours read from LDS.  The block's
// tile of the current plane (BX x BY cells) plus its x and y halos (3 cells
// each side, no corners) is staged in LDS per field; the interior comes from
// the z register window, so only the halo is fetched from memory, and each
// cell's twelve x/y neighbour loads become LDS reads.  Two tile buffers
// alternate between planes, so one barrier per plane suffices.  Requires the
// tile to divide the grid in x and y (nx % BX == 0, ny % BY == 0); the
// arithmetic is that of filter_body term by term.
template <typename T, int NF>
__device__ __forceinline__ void filter_lds_body(const FiltArgs<T>& a, const BlockIdx3& bi) {
    extern __shared__ unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    const Grid& g = a.g;
    const Col col = column(g, a.kc, bi);
    const int BX = blockDim.x, BY = blockDim.y;
    const int W = BX + 6, H = BY + 6;          // tile row length and rows
    const int tsz = W * H;                     // one field's tile
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = tx + BX * ty, nthr = BX * BY;
    const int i0 = col.i - tx, j0 = col.j - ty;   // tile origin (all columns active)
    const int lgBX = __ffs(BX) - 1;
    const unsigned nxy = (unsigned)g.nxy;
    const unsigned cell = col.row + col.i;
    const T c6 = T(INV_PI6);
    Partial part = {0, 0, 0, 0, 0, 0};
    const int dir = col.dir;
    const int k0 = col.k0, k1 = col.k1;
    const int ks = dir > 0 ? k0 : k1 - 1;
    constexpr int HM = 2;
    const HaloMap<HM> hm = halo_map<3, HM>(i0, j0, g, BX, lgBX, BY, tid, nthr);
    // Loads run one plane ahead of their use: the window's next plane (pf)
    // and the next plane's halo (hv) are fetched while this plane is computed.
    T win[NF][7], pf[NF], hv[NF][HM];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int m = 0; m < 7; ++m) win[f][m] = a.in[f][(unsigned)wrap(ks + (m - 3) * dir, g.nz) * nxy + cell];
        pf[f] = a.in[f][(unsigned)wrap(ks + 4 * dir, g.nz) * nxy + cell];
#pragma unroll
        for (int h = 0; h < HM; ++h)
            hv[f][h] = h < hm.n ? a.in[f][(unsigned)ks * nxy + hm.src[h]] : T(0);
    }
    int buf = 0;
    for (int k = ks, left = k1 - k0; left > 0; --left, k += dir, buf ^= 1) {
        const unsigned base = (unsigned)k * nxy;
        const unsigned idx = base + cell;
        T* tb = lds + buf * NF * tsz;
        // stage this plane: interior from the window, halo from the prefetch
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            tb[f * tsz + (ty + 3) * W + tx + 3] = win[f][3];
#pragma unroll
            for (int h = 0; h < HM; ++h)
                if (h < hm.n) tb[f * tsz + hm.dst[h]] = hv[f][h];
        }
        if (left > 1) {
            const unsigned nb = (unsigned)wrap(k + dir, g.nz) * nxy;
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int h = 0; h < HM; ++h)
                    if (h < hm.n) hv[f][h] = a.in[f][nb + hm.src[h]];
        }
        __syncthreads();
        const uint8_t fl = a.flags[idx];
        T res[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const T f0 = win[f][3];
            const T* rowp = tb + f * tsz + (ty + 3) * W + tx;        // rowp[m] = x offset m - 3
            const T* colp = tb + f * tsz + ty * W + tx + 3;          // colp[m W] = y offset m - 3
            const T dx6 = (rowp[0] + rowp[6]) - T(6) * (rowp[1] + rowp[5]) +
                          T(15) * (rowp[2] + rowp[4]) - T(20) * f0;
            const T dy6 = (colp[0] + colp[6 * W]) - T(6) * (colp[W] + colp[5 * W]) +
                          T(15) * (colp[2 * W] + colp[4 * W]) - T(20) * f0;
            const T dz6 = (win[f][0] + win[f][6]) - T(6) * (win[f][1] + win[f][5]) +
                          T(15) * (win[f][2] + win[f][4]) - T(20) * f0;
            res[f] = (fl & F_FLUID) ? f0 + c6 * (dx6 + dy6 + dz6) : T(0);
            a.out[f][idx] = res[f];
#pragma unroll
            for (int m = 0; m < 6; ++m) win[f][m] = win[f][m + 1];
            win[f][6] = pf[f];
            if (left > 1) pf[f] = a.in[f][(unsigned)wrap(k + 5 * dir, g.nz) * nxy + cell];
        }
        if (a.part.p) {
            const double b = (fl & F_FLUID) ? 1.0 : 0.0;
            if (NF == 3) {
                const double u = (double)res[0], v = (double)res[1], w = (double)res[2];
                part.ke += b * (u * u + v * v + w * w);
                part.rate = fmax(part.rate, courant_rate(u, v, w, g));
            } else {
                const double c = (double)res[0];
                part.mass += b * c;
                if (fl & F_ROOM) { part.room_num += b * c; part.room_den += b; }
            }
        }
    }
    if (a.part.p) block_reduce_partial<NF == 3 ? PM_VEL : PM_SCA>(part, a.part, (int)bi.hw);
}

// The LDS filter with the pair kernels' register rings (filter_lds_body's
// arithmetic, in the same order): the z window of each field, the flags and
// the x/y halo live in rings indexed by the march position, over a z loop
// unrolled U times, and every access is a raw buffer access with a scalar
// plane offset.  The tile is 64 x BY (compile time), so LDS offsets are
// immediates.
template <typename T, int NF, int BY>
__device__ __forceinline__ void filter_ring_body(const FiltArgs<T>& a, const BlockIdx3& bi) {
    constexpr int BX = 64, W = BX + 6, H = BY + 6, TSZ = W * H;
    constexpr int U = 8;                                   // window (7 planes) and its prefetch
    constexpr int HM = (6 * (BX + BY) + BX * BY - 1) / (BX * BY);
    constexpr unsigned E = sizeof(T);
    extern __shared__ unsigned char smem_raw[];
    T* const lds = reinterpret_cast<T*>(smem_raw);        // [2 planes][NF][TSZ]
    const Grid& g = a.g;
    const Col col = column(g, a.kc, bi);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + BX * ty;
    const int i0 = col.i - tx, j0 = col.j - ty;
    const unsigned cell = col.row + col.i, cb = cell * E;
    const T c6 = T(INV_PI6);
    Partial part = {0, 0, 0, 0, 0, 0};
    const int dir = col.dir, k0 = col.k0, k1 = col.k1;
    const int ks = dir > 0 ? k0 : k1 - 1;
    const int n = k1 - k0;
    const HaloMap<HM> hm = halo_map<3, HM>(i0, j0, g, BX, 6, BY, tid, BX * BY);
    unsigned hb[HM];
#pragma unroll
    for (int h = 0; h < HM; ++h) hb[h] = hm.src[h] * E;
    const int cc0 = (ty + 3) * W + tx + 3;
    const unsigned nxy = (unsigned)g.nxy, ntot = (unsigned)g.nz * nxy;
    auto pl = [&](int m) -> unsigned { return (unsigned)wrap(ks + m * dir, g.nz) * nxy; };
    auto step = [&](unsigned p) -> unsigned {
        return dir > 0 ? (p + nxy == ntot ? 0u : p + nxy) : (p == 0 ? ntot - nxy : p - nxy);
    };
    // rings by march position m (plane ks + m dir): win (the z window and
    // its prefetch, positions r-3 .. r+4 at iteration r), fq (flags), hv
    // (x/y halo, positions r and r+1)
    T win[NF][U], hv[NF][2][HM];
    uint8_t fq[U];
#pragma unroll
    for (int s = 0; s < U; ++s) {
        fq[s] = 0;
#pragma unroll
        for (int f = 0; f < NF; ++f) win[f][s] = T(0);
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int m = -3; m <= 4; ++m) win[f][(m + U) % U] = bld(a.in[f], cb, pl(m) * E);
#pragma unroll
        for (int h = 0; h < HM; ++h) {
            hv[f][0][h] = bld(a.in[f], hb[h], pl(0) * E);   // (lanes without a halo cell read cell 0)
            hv[f][1][h] = T(0);
        }
    }
    fq[0] = bld(a.flags, cell, pl(0));
    unsigned p0 = pl(0), p1 = pl(1), p5 = pl(5);   // planes of positions r, r + 1, r + 5
    int r = 0;
    auto iter = [&](auto phase) __attribute__((always_inline)) -> bool {
        constexpr int P = decltype(phase)::value;
        constexpr int B = P & 1;
        if (r >= n) return false;
        const int cc = opaque(cc0);
        int hd[HM];
#pragma unroll
        for (int h = 0; h < HM; ++h) hd[h] = opaque(hm.dst[h]);
        T* const tb = lds + B * NF * TSZ;
        // stage this plane: interior from the window, halo from the prefetch
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            tb[f * TSZ + cc] = win[f][P % U];
#pragma unroll
            for (int h = 0; h < HM; ++h)
                if (h < hm.n) tb[f * TSZ + hd[h]] = hv[f][B][h];
        }
        // the next plane's halo and flags; on the chunk's last plane the
        // loads still run, from this plane (valid memory, never used), so that
        // no branch, and no select that the compiler could fold into the
        // flag tests (which would wait for the load at once), is needed
        const bool more = r + 1 < n;
        const unsigned q1 = more ? p1 : p0, q5 = more ? p5 : p0;
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int h = 0; h < HM; ++h) hv[f][B ^ 1][h] = bld(a.in[f], hb[h], q1 * E);
        fq[(P + 1) % U] = bld(a.flags, cell, q1);
        __syncthreads();
        const uint8_t fl = fq[P % U];
        T res[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const T f0 = win[f][P % U];
            const T* rowp = tb + f * TSZ + cc - 3;        // rowp[m] = x offset m - 3
            const T* colp = tb + f * TSZ + cc - 3 * W;    // colp[m W] = y offset m - 3
            const T dx6 = (rowp[0] + rowp[6]) - T(6) * (rowp[1] + rowp[5]) +
                          T(15) * (rowp[2] + rowp[4]) - T(20) * f0;
            const T dy6 = (colp[0] + colp[6 * W]) - T(6) * (colp[W] + colp[5 * W]) +
                          T(15) * (colp[2 * W] + colp[4 * W]) - T(20) * f0;
            const T dz6 = (win[f][(P + U - 3) % U] + win[f][(P + 3) % U]) -
                          T(6) * (win[f][(P + U - 2) % U] + win[f][(P + 2) % U]) +
                          T(15) * (win[f][(P + U - 1) % U] + win[f][(P + 1) % U]) - T(20) * f0;
            res[f] = (fl & F_FLUID) ? f0 + c6 * (dx6 + dy6 + dz6) : T(0);
            bst(a.out[f], cb, p0 * E, res[f]);
            // the window's next plane (position r + 5, into the slot of r - 3)
            win[f][(P + 5) % U] = bld(a.in[f], cb, q5 * E);
        }
        if (a.part.p) {
            const double b = (fl & F_FLUID) ? 1.0 : 0.0;
            if (NF == 3) {
                const double u = (double)res[0], v = (double)res[1], w = (double)res[2];
                part.ke += b * (u * u + v * v + w * w);
                part.rate = fmax(part.rate, courant_rate(u, v, w, g));
            } else {
                const double c = (double)res[0];
                part.mass += b * c;
                if (fl & F_ROOM) { part.room_num += b * c; part.room_den += b; }
            }
        }
        p0 = step(p0);
        p1 = step(p1);
        p5 = step(p5);
        ++r;
        return true;
    };
    while (pair_phases(std::make_integer_sequence<int, U>{}, iter)) {
    }
    if (a.part.p) block_reduce_partial<NF == 3 ? PM_VEL : PM_SCA>(part, a.part, (int)bi.hw);
}

// ---------------------------------------------------------------------------
// Velocity correction of Section 2.2 with the mask: out = beta (u* - grad p).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void correct_body(const CorrArgs<T>& a, const BlockIdx3& bi) {
    const Grid& g = a.g;
    const Col col = column(g, a.kc, bi);
    Partial part = {0, 0, 0, 0, 0, 0};
    if (col.active) {
        const int k0 = col.k0, k1 = col.k1;
        const unsigned nxy = (unsigned)g.nxy;
        const T hx = T(g.inv2d[0]), hy = T(g.inv2d[1]), hz = T(g.inv2d[2]);
        const T* __restrict__ p = a.p;
        T pm = p[(unsigned)(k0 == 0 ? g.nz - 1 : k0 - 1) * nxy + col.row + col.i];
        T p0 = p[(unsigned)k0 * nxy + col.row + col.i];
        for (int k = k0; k < k1; ++k) {
            const int kp = k + 1 == g.nz ? 0 : k + 1;
            const unsigned base = (unsigned)k * nxy;
            const unsigned idx = base + col.row + col.i;
            const T pp = p[(unsigned)kp * nxy + col.row + col.i];
            const T gx = (p[base + col.row + col.ip] - p[base + col.row + col.im]) * hx;
            const T gy = (p[base + col.rowp + col.i] - p[base + col.rowm + col.i]) * hy;
            const T gz = (pp - pm) * hz;
            const bool fluid = a.flags[idx] & F_FLUID;
            const T u = a.us[0][idx], v = a.us[1][idx], w = a.us[2][idx];
            const T uo = fluid ? u - gx : T(0), vo = fluid ? v - gy : T(0), wo = fluid ? w - gz : T(0);
            a.out[0][idx] = uo;
            a.out[1][idx] = vo;
            a.out[2][idx] = wo;
            if (a.part.p) {
                const double ud = (double)uo, vd = (double)vo, wd = (double)wo;
                part.ke += fluid ? ud * ud + vd * vd + wd * wd : 0.0;
                part.rate = fmax(part.rate, courant_rate(ud, vd, wd, g));
            }
            pm = p0; p0 = pp;
        }
    }
    if (a.part.p) block_reduce_partial<PM_VEL>(part, a.part, (int)bi.hw);
}

// Velocity correction (correct_body, or refine_correct_body when REFINE: the
// pressure is p4 + dp in FP64 and is written back) as a register-ring march
// over 64 x BY tiles: the pressure of each plane is staged in LDS with its
// one-cell x/y halo, its z neighbours come from a ring, the next plane's
// u*, flags and halo and the pressure two planes ahead are in flight while a
// plane is corrected, and every access is a raw buffer access with a scalar
// plane offset.  Same arithmetic as the plain kernels.
template <typename T, bool REFINE>
struct CorrRingIO;
template <typename T>
struct CorrRingIO<T, false> {
    using Q = T;
    const T* p;
    __device__ __forceinline__ Q q(unsigned voff, unsigned plane) const { return bld(p, voff * sizeof(T), plane * sizeof(T)); }
};
template <typename T>
struct CorrRingIO<T, true> {
    using Q = double;
    const float* p4;
    const float* dp;
    __device__ __forceinline__ Q q(unsigned voff, unsigned plane) const {
        return (double)bld(p4, voff * 4u, plane * 4u) + (double)bld(dp, voff * 4u, plane * 4u);
    }
};
template <typename T, bool REFINE, int BY, int D>
__device__ __forceinline__ void correct_ring_body(const T* const us[3], T* const out[3], const CorrRingIO<T, REFINE> io,
                                                  float* pout, const uint8_t* flags, const Grid& g, int kc,
                                                  const PartSoA& pa, const BlockIdx3& bi) {
    using Q = typename CorrRingIO<T, REFINE>::Q;
    constexpr int BX = 64, W = BX + 2, TS = W * (BY + 2);
    constexpr int U = (D + 4) & ~1;                     // even, >= D + 3
    constexpr int HM = (2 * (BX + BY) + BX * BY - 1) / (BX * BY);
    constexpr unsigned E = sizeof(T);
    extern __shared__ unsigned char smem_raw[];
    Q* const lds = reinterpret_cast<Q*>(smem_raw);     // [2 planes][TS]
    const Col col = column(g, kc, bi);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + BX * ty;
    const int i0 = col.i - tx, j0 = col.j - ty;
    const unsigned cell = col.row + col.i, cb = cell * E;
    const int k0 = col.k0, k1 = col.k1, n = k1 - k0;
    const HaloMap<HM> hm = halo_map<1, HM>(i0, j0, g, BX, 6, BY, tid, BX * BY);
    const int cc0 = (ty + 1) * W + tx + 1;
    const unsigned nxy = (unsigned)g.nxy, ntot = (unsigned)g.nz * nxy;
    auto pl = [&](int k) -> unsigned { return (unsigned)wrap(k, g.nz) * nxy; };
    auto step = [&](unsigned p) -> unsigned { return p + nxy == ntot ? 0u : p + nxy; };
    Partial part = {0, 0, 0, 0, 0, 0};
    // rings by plane position m (plane k0 + m): pz (pressure at the cell,
    // positions r-1 .. r+1+D), uq and fq (u* and flags, r .. r+D), hv (the
    // pressure halo, r .. r+D); loads run D planes ahead
    Q pz[U], hv[U][HM];
    T uq[U][3];
    uint8_t fq[U];
#pragma unroll
    for (int s = 0; s < U; ++s) {
        pz[s] = Q(0);
        fq[s] = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) uq[s][c] = T(0);
#pragma unroll
        for (int h = 0; h < HM; ++h) hv[s][h] = Q(0);
    }
#pragma unroll
    for (int m = -1; m <= D; ++m) pz[(m + U) % U] = io.q(cell, pl(k0 + m));
#pragma unroll
    for (int m = 0; m < D; ++m) {
        const unsigned pm = pl(k0 + m);
#pragma unroll
        for (int c = 0; c < 3; ++c) uq[m][c] = bld(us[c], cb, pm * E);
        fq[m] = bld(flags, cell, pm);
#pragma unroll
        for (int h = 0; h < HM; ++h) hv[m][h] = io.q(hm.src[h], pm);   // (lanes without a halo cell read cell 0)
    }
    unsigned p0 = pl(k0), pd = pl(k0 + D), pd1 = pl(k0 + D + 1);
    int r = 0;
    auto iter = [&](auto phase) __attribute__((always_inline)) -> bool {
        constexpr int P = decltype(phase)::value;
        constexpr int B = P & 1;
        if (r >= n) return false;
        const int cc = opaque(cc0);
        int hd[HM];
#pragma unroll
        for (int h = 0; h < HM; ++h) hd[h] = opaque(hm.dst[h]);
        Q* const tb = lds + B * TS;
        tb[cc] = pz[P % U];
#pragma unroll
        for (int h = 0; h < HM; ++h)
            if (h < hm.n) tb[hd[h]] = hv[P % U][h];
        // u*, flags and halo of plane r + D, the pressure of plane r + 1 + D
        // (past the chunk's end from this plane: valid memory, never used)
        const bool more = r + D < n;
        const unsigned q1 = more ? pd : p0, q2 = more ? pd1 : p0;
#pragma unroll
        for (int h = 0; h < HM; ++h) hv[(P + D) % U][h] = io.q(hm.src[h], q1);
        pz[(P + 1 + D) % U] = io.q(cell, q2);
#pragma unroll
        for (int c = 0; c < 3; ++c) uq[(P + D) % U][c] = bld(us[c], cb, q1 * E);
        fq[(P + D) % U] = bld(flags, cell, q1);
        __syncthreads();
        const bool fluid = fq[P % U] & F_FLUID;
        const Q gx = (tb[cc + 1] - tb[cc - 1]) * Q(g.inv2d[0]);
        const Q gy = (tb[cc + W] - tb[cc - W]) * Q(g.inv2d[1]);
        const Q gz = (pz[(P + 1) % U] - pz[(P + U - 1) % U]) * Q(g.inv2d[2]);
        T o[3];
        if (REFINE) {
            const double u = uq[P % U][0], v = uq[P % U][1], w = uq[P % U][2];
            o[0] = fluid ? (T)(u - gx) : T(0);
            o[1] = fluid ? (T)(v - gy) : T(0);
            o[2] = fluid ? (T)(w - gz) : T(0);
            bst(pout, cell * 4u, p0 * 4u, (float)pz[P % U]);
        } else {
            o[0] = fluid ? uq[P % U][0] - (T)gx : T(0);
            o[1] = fluid ? uq[P % U][1] - (T)gy : T(0);
            o[2] = fluid ? uq[P % U][2] - (T)gz : T(0);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) bst(out[c], cb, p0 * E, o[c]);
        if (pa.p) {
            const double ud = (double)o[0], vd = (double)o[1], wd = (double)o[2];
            part.ke += fluid ? ud * ud + vd * vd + wd * wd : 0.0;
            part.rate = fmax(part.rate, courant_rate(ud, vd, wd, g));
        }
        p0 = step(p0);
        pd = step(pd);
        pd1 = step(pd1);
        ++r;
        return true;
    };
    while (pair_phases(std::make_integer_sequence<int, U>{}, iter)) {
    }
    if (pa.p) block_reduce_partial<PM_VEL>(part, pa, (int)bi.hw);
}

// ---------------------------------------------------------------------------
// FP64 residual of the last FP32 pressure solve (iterative refinement):
// res = div u* + div((1-beta) grad p3) - div grad p4, all in FP64.  The
// radius-2 operator div grad p4 = sum_a (p4(x+2e) - 2 p4 + p4(x-2e)) / (4 dx_a^2).
// The dense kernel writes the cells without a solid face neighbour (no IB
// term); the cells of the immersed-boundary list, whose IB term needs the
// solid neighbours and p3, get their whole residual from a sparse kernel
// over that list, so the dense march carries no gathers that depend on
// loaded flags.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void refine_res_body(const RefineResArgs& a, const BlockIdx3& bi) {
    const Grid& g = a.g;
    const Col col = column(g, a.kc, bi);
    if (!col.active) return;
    const int k0 = col.k0, k1 = col.k1;
    const unsigned nxy = (unsigned)g.nxy;
    const int ixm2 = wrap(col.i - 2, g.nx), ixp2 = wrap(col.i + 2, g.nx);
    const unsigned rowm2 = (unsigned)wrap(col.j - 2, g.ny) * g.nx, rowp2 = (unsigned)wrap(col.j + 2, g.ny) * g.nx;
    const double h2[3] = {g.inv2d[0], g.inv2d[1], g.inv2d[2]};
    // z windows: w at k-1..k+1, p4 at k-2..k+2
    double wz[3], pz[5];
#pragma unroll
    for (int m = 0; m < 2; ++m) wz[m] = (double)a.us[2][(unsigned)wrap(k0 - 1 + m, g.nz) * nxy + col.row + col.i];
#pragma unroll
    for (int m = 0; m < 4; ++m) pz[m] = (double)a.p4[(unsigned)wrap(k0 - 2 + m, g.nz) * nxy + col.row + col.i];
    for (int k = k0; k < k1; ++k) {
        const unsigned base = (unsigned)k * nxy;
        const unsigned idx = base + col.row + col.i;
        wz[2] = (double)a.us[2][(unsigned)wrap(k + 1, g.nz) * nxy + col.row + col.i];
        pz[4] = (double)a.p4[(unsigned)wrap(k + 2, g.nz) * nxy + col.row + col.i];
        const double div = ((double)a.us[0][base + col.row + col.ip] - (double)a.us[0][base + col.row + col.im]) * h2[0] +
                           ((double)a.us[1][base + col.rowp + col.i] - (double)a.us[1][base + col.rowm + col.i]) * h2[1] +
                           (wz[2] - wz[0]) * h2[2];
        const double p0 = pz[2];
        const double lap =
            ((double)a.p4[base + col.row + ixp2] - 2.0 * p0 + (double)a.p4[base + col.row + ixm2]) * (h2[0] * h2[0]) +
            ((double)a.p4[base + rowp2 + col.i] - 2.0 * p0 + (double)a.p4[base + rowm2 + col.i]) * (h2[1] * h2[1]) +
            (pz[4] - 2.0 * p0 + pz[0]) * (h2[2] * h2[2]);
        if (!(a.flags[idx] & F_NEAR_SOLID)) a.res[idx] = (float)(div - lap);
        wz[0] = wz[1]; wz[1] = wz[2];
#pragma unroll
        for (int m = 0; m < 4; ++m) pz[m] = pz[m + 1];
    }
}

// The listed cells: div u* - div grad p4 as in the dense kernel, plus
// div((1-beta) grad p3) from the faces whose neighbour is solid (mask bits
// +x, -x, +y, -y, +z, -z = 1, 2, 4, 8, 16, 32).
__device__ __forceinline__ void refine_res_ib_body(const RefineResArgs& a, unsigned blk) {
    const int e = blk * blockDim.x + threadIdx.x;
    if (e >= a.ib.n) return;
    const Grid& g = a.g;
    const unsigned idx = (unsigned)a.ib.idx[e];
    const unsigned mask = a.ib.mask[e];
    const unsigned nx = g.nx, ny = g.ny, nz = g.nz, nxy = nx * ny;
    const unsigned i = idx % nx, jk = idx / nx;
    const unsigned j = jk % ny, k = jk / ny;
    auto sx = [&](int d) { return idx - i + (unsigned)wrap((int)i + d, (int)nx); };
    auto sy = [&](int d) { return idx + ((unsigned)wrap((int)j + d, (int)ny) - j) * nx; };
    auto sz = [&](int d) { return idx + ((unsigned)wrap((int)k + d, (int)nz) - k) * nxy; };
    const double h2[3] = {g.inv2d[0], g.inv2d[1], g.inv2d[2]};
    const double div = ((double)a.us[0][sx(1)] - (double)a.us[0][sx(-1)]) * h2[0] +
                       ((double)a.us[1][sy(1)] - (double)a.us[1][sy(-1)]) * h2[1] +
                       ((double)a.us[2][sz(1)] - (double)a.us[2][sz(-1)]) * h2[2];
    const double p0 = (double)a.p4[idx];
    const double lap = ((double)a.p4[sx(2)] - 2.0 * p0 + (double)a.p4[sx(-2)]) * (h2[0] * h2[0]) +
                       ((double)a.p4[sy(2)] - 2.0 * p0 + (double)a.p4[sy(-2)]) * (h2[1] * h2[1]) +
                       ((double)a.p4[sz(2)] - 2.0 * p0 + (double)a.p4[sz(-2)]) * (h2[2] * h2[2]);
    const double q0 = (double)a.p3[idx];
    double ib = 0.0;
    if (mask & 1u) ib += (((double)a.p3[sx(2)] - q0) * h2[0]) * h2[0];
    if (mask & 2u) ib -= ((q0 - (double)a.p3[sx(-2)]) * h2[0]) * h2[0];
    if (mask & 4u) ib += (((double)a.p3[sy(2)] - q0) * h2[1]) * h2[1];
    if (mask & 8u) ib -= ((q0 - (double)a.p3[sy(-2)]) * h2[1]) * h2[1];
    if (mask & 16u) ib += (((double)a.p3[sz(2)] - q0) * h2[2]) * h2[2];
    if (mask & 32u) ib -= ((q0 - (double)a.p3[sz(-2)]) * h2[2]) * h2[2];
    a.res[idx] = (float)(div + ib - lap);
}

// u = beta (u* - grad(p4 + dp)), p = p4 + dp, FP64 arithmetic, FP32 storage.
__device__ __forceinline__ void refine_correct_body(const RefineCorrArgs& a, const BlockIdx3& bi) {
    const Grid& g = a.g;
    const Col col = column(g, a.kc, bi);
    Partial part = {0, 0, 0, 0, 0, 0};
    if (col.active) {
        const int k0 = col.k0, k1 = col.k1;
        const unsigned nxy = (unsigned)g.nxy;
        auto P = [&](unsigned i) -> double { return (double)a.p4[i] + (double)a.dp[i]; };
        double qm = P((unsigned)wrap(k0 - 1, g.nz) * nxy + col.row + col.i);
        double q0 = P((unsigned)k0 * nxy + col.row + col.i);
        for (int k = k0; k < k1; ++k) {
            const unsigned base = (unsigned)k * nxy;
            const unsigned idx = base + col.row + col.i;
            const double qp = P((unsigned)wrap(k + 1, g.nz) * nxy + col.row + col.i);
            const double gx = (P(base + col.row + col.ip) - P(base + col.row + col.im)) * g.inv2d[0];
            const double gy = (P(base + col.rowp + col.i) - P(base + col.rowm + col.i)) * g.inv2d[1];
            const double gz = (qp - qm) * g.inv2d[2];
            const bool fluid = a.flags[idx] & F_FLUID;
            const double u = a.us[0][idx], v = a.us[1][idx], w = a.us[2][idx];
            const float uo = fluid ? (float)(u - gx) : 0.0f;
            const float vo = fluid ? (float)(v - gy) : 0.0f;
            const float wo = fluid ? (float)(w - gz) : 0.0f;
            a.out[0][idx] = uo;
            a.out[1][idx] = vo;
            a.out[2][idx] = wo;
            a.p[idx] = (float)q0;
            if (a.part.p) {
                const double ud = (double)uo, vd = (double)vo, wd = (double)wo;
                part.ke += fluid ? ud * ud + vd * vd + wd * wd : 0.0;
                part.rate = fmax(part.rate, courant_rate(ud, vd, wd, g));
            }
            qm = q0; q0 = qp;
        }
    }
    if (a.part.p) block_reduce_partial<PM_VEL>(part, a.part, (int)bi.hw);
}

// Divergence with central differences: out = sum_a D_a u_a (Section 2.2).
template <typename T>
__device__ __forceinline__ void div_body(const DivArgs<T>& a, const BlockIdx3& bi) {
    const Grid& g = a.g;
    const Col col = column(g, a.kc, bi);
    if (!col.active) return;
    const int k0 = col.k0, k1 = col.k1;
    const unsigned nxy = (unsigned)g.nxy;
    const T hx = T(g.inv2d[0]), hy = T(g.inv2d[1]), hz = T(g.inv2d[2]);
    const T* __restrict__ w = a.u[2];
    T wm = w[(unsigned)(k0 == 0 ? g.nz - 1 : k0 - 1) * nxy + col.row + col.i];
    T w0 = w[(unsigned)k0 * nxy + col.row + col.i];
    for (int k = k0; k < k1; ++k) {
        const int kp = k + 1 == g.nz ? 0 : k + 1;
        const unsigned base = (unsigned)k * nxy;
        const unsigned idx = base + col.row + col.i;
        const T wp = w[(unsigned)kp * nxy + col.row + col.i];
        const T dx = (a.u[0][base + col.row + col.ip] - a.u[0][base + col.row + col.im]) * hx;
        const T dy = (a.u[1][base + col.rowp + col.i] - a.u[1][base + col.rowm + col.i]) * hy;
        a.out[idx] = dx + dy + (wp - wm) * hz;
        wm = w0; w0 = wp;
    }
}

// Courant rate partials (max over cells), for the first step after (re)binding.
template <typename T>
__global__ __launch_bounds__(1024) void k_rate(const T* u, const T* v, const T* w, const Grid g, int kc,
                                              PartSoA part) {
    const BlockIdx3 bi = hw_block();
    const Col col = column(g, kc, bi);
    const int k0 = col.k0, k1 = col.k1;
    Partial pp = {0, 0, 0, 0, 0, 0};
    if (col.active) {
        for (int k = k0; k < k1; ++k) {
            const unsigned idx = (unsigned)k * (unsigned)g.nxy + col.row + col.i;
            pp.rate = fmax(pp.rate, courant_rate((double)u[idx], (double)v[idx], (double)w[idx], g));
        }
    }
    block_reduce_partial<PM_RATE>(pp, part, (int)bi.hw);
}

__device__ inline double next_dt(const StepScalars& s, double rate) {
    return s.dt_fixed > 0 ? s.dt_fixed : s.cfl / fmax(rate, s.rate_floor);
}

// One block: sum (or max) field f of the partials of n blocks in a fixed
// order.  Each thread takes blocks tid, tid + nthr, ... four loads at a time;
// the per-thread results are combined by block_reduce_partial.
__device__ __forceinline__ double gather_partial(PartSoA part, int f, int n, bool is_max) {
    const double* __restrict__ q = part.p + (size_t)f * part.stride;
    const int nthr = blockDim.x;
    constexpr int U = 4;
    double acc = 0.0;
    for (int b0 = threadIdx.x; b0 < n; b0 += U * nthr) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + u * nthr;
            v[u] = b < n ? q[b] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc = is_max ? fmax(acc, v[u]) : acc + v[u];
    }
    return acc;
}

// Velocity side of the end of a step: the new velocity's Courant rate gives
// the next dt; t and the step count advance by the step just taken, whose dt
// and starting rate are kept for its diagnostics record.
__device__ __forceinline__ void advance_body(const AdvanceArgs& a) {
    Partial acc = {0, 0, 0, 0, 0, 0};
    acc.rate = gather_partial(a.part, PF_RATE, a.np, true);
    __shared__ double res[PF_COUNT];
    PartSoA sh = {res, 1};
    block_reduce_partial<PM_RATE>(acc, sh, 0);
    __syncthreads();
    if (threadIdx.x == 0) {
        StepScalars* sc = a.sc;
        const double rate = res[PF_RATE];
        const double dt = sc->dt;
        sc->last_dt = dt;
        sc->last_rate = sc->rate;
        sc->t = sc->t + dt;
        sc->step = sc->step + 1;
        sc->rate = rate;
        sc->dt = next_dt(*sc, rate);
        if (!isfinite(rate)) sc->nonfinite = 1;
    }
}

// Diagnostics record of the step just advanced (after advance_body): kinetic
// energy, divergence norm, CO2 mass and room mean from the partials.
__device__ __forceinline__ void diag_body(const DiagArgs& a) {
    Partial acc = {0, 0, 0, 0, 0, 0};
    acc.ke = gather_partial(a.part, PF_KE, a.np_vel, false);
    acc.mass = gather_partial(a.part, PF_MASS, a.np_sca, false);
    acc.room_num = gather_partial(a.part, PF_RNUM, a.np_sca, false);
    acc.room_den = gather_partial(a.part, PF_RDEN, a.np_sca, false);
    acc.div2 = gather_partial(a.part, PF_DIV2, a.np_div, false);
    __shared__ double res[PF_COUNT];
    PartSoA sh = {res, 1};
    block_reduce_partial<PM_SCA | PM_DIV | (1 << PF_KE)>(acc, sh, 0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const StepScalars* sc = a.sc;
        DiagRec d;
        d.dt = sc->last_dt;
        d.t = sc->t;
        d.step = sc->step;
        d.ke = 0.5 * res[PF_KE] * a.dv;
        d.div_l2 = sqrt(res[PF_DIV2] * a.dv);
        d.co2_mass = res[PF_MASS] * a.dv;
        d.co2_room_mean = res[PF_RDEN] > 0 ? res[PF_RNUM] / res[PF_RDEN] : 0.0;
        d.cfl_max = d.dt * sc->last_rate;
        const bool bad = !isfinite(d.ke) || !isfinite(d.co2_mass) || !isfinite(d.div_l2);
        if (bad) a.sc->nonfinite_diag = 1;
        a.ring[(d.step - 1) % a.ring_cap] = d;
    }
}

// Rate only (first step after binding a state): sets the rate and the next dt.
__global__ __launch_bounds__(1024) void k_set_rate(PartSoA part, int np, StepScalars* sc) {
    Partial acc = {0, 0, 0, 0, 0, 0};
    acc.rate = gather_partial(part, PF_RATE, np, true);
    __shared__ double res[PF_COUNT];
    PartSoA sh = {res, 1};
    block_reduce_partial<PM_RATE>(acc, sh, 0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double rate = res[PF_RATE];
        sc->rate = rate;
        sc->dt = next_dt(*sc, rate);
        if (!isfinite(rate)) sc->nonfinite = 1;
    }
}


// ---------------------------------------------------------------------------
// Launch wrappers: a plain launch (block coordinates from the hardware) and a
// batched launch over several scenarios (coordinates from a table; each
// scenario's blocks compute exactly what its plain launch would).
// ---------------------------------------------------------------------------
#define DNSLAB_BATCH_COORD(tab, st, ns)                 \
    const int s_ = batch_slot(st, ns);                  \
    BlockIdx3 bi_;                                      \
    bi_.hw = blockIdx.x - st[s_];                       \
    bi_.gx = tab[s_].g[0];                              \
    bi_.gy = tab[s_].g[1];                              \
    bi_.gz = tab[s_].g[2];

template <typename T, int MODE, bool LDS>
__global__ __launch_bounds__(1024) void k_mom_stage(const MomArgs<T> a) { mom_stage_body<T, MODE, LDS>(a, hw_block()); }
template <typename T, int MODE, bool LDS>
__global__ __launch_bounds__(1024) void k_mom_stage_b(const BRec<MomArgs<T>>* __restrict__ tab,
                                                      const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    const MomArgs<T> a = tab[s_].a;
    mom_stage_body<T, MODE, LDS>(a, bi_);
}
template <typename T, int PAIR>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(pair_waves<T, true, PAIR>()))) void k_mom_pair(const MomPairArgs<T> a) {
    mom_pair_body<T, PAIR, pair_dist<T, true, PAIR>(), DNSLAB_PROWS>(a, hw_block());
}
template <typename T, int PAIR>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(pair_waves<T, true, PAIR>()))) void k_mom_pair_b(const BRec<MomPairArgs<T>>* __restrict__ tab,
                                                    const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    const MomPairArgs<T> a = tab[s_].a;
    mom_pair_body<T, PAIR, pair_dist<T, true, PAIR>(), DNSLAB_PROWS>(a, bi_);
}
template <typename T, int PAIR>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(pair_waves<T, false, PAIR>()))) void k_sca_pair(const ScaPairArgs<T> a) {
    sca_pair_body<T, PAIR, pair_dist<T, false, PAIR>(), DNSLAB_PROWS>(a, hw_block());
}
template <typename T, int PAIR>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(pair_waves<T, false, PAIR>()))) void k_sca_pair_b(const BRec<ScaPairArgs<T>>* __restrict__ tab,
                                                    const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    const ScaPairArgs<T> a = tab[s_].a;
    sca_pair_body<T, PAIR, pair_dist<T, false, PAIR>(), DNSLAB_PROWS>(a, bi_);
}
template <typename T, int MODE>
__global__ __launch_bounds__(1024) void k_sca_stage(const ScaArgs<T> a) { sca_stage_body<T, MODE>(a, hw_block()); }
template <typename T, int MODE>
__global__ __launch_bounds__(1024) void k_sca_stage_b(const BRec<ScaArgs<T>>* __restrict__ tab,
                                                      const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    const ScaArgs<T> a = tab[s_].a;
    sca_stage_body<T, MODE>(a, bi_);
}
template <typename T, int NF>
__global__ __launch_bounds__(1024) void k_filter(const FiltArgs<T> a) { filter_body<T, NF>(a, hw_block()); }
template <typename T, int NF>
__global__ __launch_bounds__(1024) void k_filter_b(const BRec<FiltArgs<T>>* __restrict__ tab,
                                                   const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    const FiltArgs<T> a = tab[s_].a;
    filter_body<T, NF>(a, bi_);
}
template <typename T, int NF>
__global__ __launch_bounds__(1024) void k_filter_lds(const FiltArgs<T> a) { filter_lds_body<T, NF>(a, hw_block()); }
template <typename T, int NF>
__global__ __launch_bounds__(1024) void k_filter_lds_b(const BRec<FiltArgs<T>>* __restrict__ tab,
                                                       const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    const FiltArgs<T> a = tab[s_].a;
    filter_lds_body<T, NF>(a, bi_);
}
template <typename T, int NF>
__global__ __launch_bounds__(64 * DNSLAB_FROWS) void k_filter_ring(const FiltArgs<T> a) {
    filter_ring_body<T, NF, DNSLAB_FROWS>(a, hw_block());
}
template <typename T, int NF>
__global__ __launch_bounds__(64 * DNSLAB_FROWS) void k_filter_ring_b(const BRec<FiltArgs<T>>* __restrict__ tab,
                                                       const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    const FiltArgs<T> a = tab[s_].a;
    filter_ring_body<T, NF, DNSLAB_FROWS>(a, bi_);
}
template <typename T>
__global__ __launch_bounds__(1024) void k_correct(const CorrArgs<T> a) { correct_body<T>(a, hw_block()); }
template <typename T>
__global__ __launch_bounds__(1024) void k_correct_b(const BRec<CorrArgs<T>>* __restrict__ tab,
                                                    const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    const CorrArgs<T> a = tab[s_].a;
    correct_body<T>(a, bi_);
}
template <typename T>
__global__ __launch_bounds__(1024) void k_div(const DivArgs<T> a) { div_body<T>(a, hw_block()); }
template <typename T>
__global__ __launch_bounds__(1024) void k_div_b(const BRec<DivArgs<T>>* __restrict__ tab,
                                                const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    const DivArgs<T> a = tab[s_].a;
    div_body<T>(a, bi_);
}
__global__ __launch_bounds__(1024) void k_refine_res(const RefineResArgs a) { refine_res_body(a, hw_block()); }
__global__ __launch_bounds__(1024) void k_refine_res_b(const BRec<RefineResArgs>* __restrict__ tab,
                                                       const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    const RefineResArgs a = tab[s_].a;
    refine_res_body(a, bi_);
}
__global__ __launch_bounds__(256) void k_refine_res_ib(const RefineResArgs a) { refine_res_ib_body(a, blockIdx.x); }
__global__ __launch_bounds__(256) void k_refine_res_ib_b(const BRec<RefineResArgs>* __restrict__ tab,
                                                         const unsigned* __restrict__ st, int ns) {
    const int s_ = batch_slot(st, ns);
    const RefineResArgs a = tab[s_].a;
    refine_res_ib_body(a, blockIdx.x - st[s_]);
}
template <typename T>
__device__ __forceinline__ void correct_ring(const CorrArgs<T>& a, const BlockIdx3& bi) {
    CorrRingIO<T, false> io;
    io.p = a.p;
    correct_ring_body<T, false, DNSLAB_FROWS, DNSLAB_RING_DIST>(a.us, a.out, io, nullptr, a.flags, a.g, a.kc, a.part, bi);
}
__device__ __forceinline__ void refine_correct_ring(const RefineCorrArgs& a, const BlockIdx3& bi) {
    CorrRingIO<float, true> io;
    io.p4 = a.p4;
    io.dp = a.dp;
    correct_ring_body<float, true, DNSLAB_FROWS, DNSLAB_RING_DIST>(a.us, a.out, io, a.p, a.flags, a.g, a.kc, a.part, bi);
}
template <typename T>
__global__ __launch_bounds__(64 * DNSLAB_FROWS) void k_correct_ring(const CorrArgs<T> a) { correct_ring<T>(a, hw_block()); }
template <typename T>
__global__ __launch_bounds__(64 * DNSLAB_FROWS) void k_correct_ring_b(const BRec<CorrArgs<T>>* __restrict__ tab,
                                                        const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    const CorrArgs<T> a = tab[s_].a;
    correct_ring<T>(a, bi_);
}
__global__ __launch_bounds__(64 * DNSLAB_FROWS) void k_refine_correct_ring(const RefineCorrArgs a) {
    refine_correct_ring(a, hw_block());
}
__global__ __launch_bounds__(64 * DNSLAB_FROWS) void k_refine_correct_ring_b(const BRec<RefineCorrArgs>* __restrict__ tab,
                                                               const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    const RefineCorrArgs a = tab[s_].a;
    refine_correct_ring(a, bi_);
}
__global__ __launch_bounds__(1024) void k_refine_correct(const RefineCorrArgs a) {
    refine_correct_body(a, hw_block());
}
__global__ __launch_bounds__(1024) void k_refine_correct_b(const BRec<RefineCorrArgs>* __restrict__ tab,
                                                           const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    const RefineCorrArgs a = tab[s_].a;
    refine_correct_body(a, bi_);
}
__global__ __launch_bounds__(1024) void k_advance(const AdvanceArgs a) { advance_body(a); }
__global__ __launch_bounds__(1024) void k_advance_b(const BRec<AdvanceArgs>* __restrict__ tab,
                                                    const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    (void)bi_;
    const AdvanceArgs a = tab[s_].a;
    advance_body(a);
}
__global__ __launch_bounds__(1024) void k_diag(const DiagArgs a) { diag_body(a); }
__global__ __launch_bounds__(1024) void k_diag_b(const BRec<DiagArgs>* __restrict__ tab,
                                                 const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_COORD(tab, st, ns)
    (void)bi_;
    const DiagArgs a = tab[s_].a;
    diag_body(a);
}

}  // namespace

StencilLaunch stencil_launch(const Grid& g, int rows, int kc, int cells_x) {
    StencilLaunch L;
    const int nxt = g.nx / cells_x;          // threads needed along x
    int bx = nxt >= 64 ? 64 : (nxt >= 32 ? 32 : 16);
    int by = std::max(1, std::min(rows * 64 / bx, 1024 / bx));
    L.block = dim3(bx, by, 1);
    L.kc = kc < 1 ? 1 : kc;
    L.grid = dim3((nxt + bx - 1) / bx, (g.ny + by - 1) / by, (g.nz + L.kc - 1) / L.kc);
    L.nblocks = (int)(L.grid.x * L.grid.y * L.grid.z);
    return L;
}


// The register-ring correction: 64 x DNSLAB_FROWS tiles dividing the grid.
inline bool correct_ring_fits(const Grid& g, const StencilLaunch& L) {
    return DNSLAB_CORRECT_RING && L.block.x == 64 && L.block.y == DNSLAB_FROWS && g.nx % 64 == 0 &&
           g.ny % DNSLAB_FROWS == 0;
}

// LDS variants of the z-marching kernels need the block's tile inside the grid.
// radius: the halo width; every thread loads at most two halo cells per field.
inline bool tile_divides(const Grid& g, const StencilLaunch& L, int radius) {
    const int bx = (int)L.block.x, by = (int)L.block.y;
    return g.nx % bx == 0 && g.ny % by == 0 && 2 * radius * (bx + by) <= 2 * bx * by;
}

template <typename T, bool LDS>
void launch_mom_modes(int mode, const MomArgs<T>& b, const StencilLaunch& L, size_t lds, hipStream_t s) {
    switch (mode) {
        case ST_FIRST: hipLaunchKernelGGL((k_mom_stage<T, ST_FIRST, LDS>), L.grid, L.block, lds, s, b); break;
        case ST_HALF: hipLaunchKernelGGL((k_mom_stage<T, ST_HALF, LDS>), L.grid, L.block, lds, s, b); break;
        case ST_FULL: hipLaunchKernelGGL((k_mom_stage<T, ST_FULL, LDS>), L.grid, L.block, lds, s, b); break;
        case ST_LAST: hipLaunchKernelGGL((k_mom_stage<T, ST_LAST, LDS>), L.grid, L.block, lds, s, b); break;
        default: hipLaunchKernelGGL((k_mom_stage<T, ST_RHS, LDS>), L.grid, L.block, lds, s, b); break;
    }
}

template <typename T>
hipError_t launch_mom_stage(int mode, const MomArgs<T>& a, const StencilLaunch& L, hipStream_t s, Recorder* rec) {
    MomArgs<T> b = a;
    b.kc = L.kc;
    const bool use_lds = DNSLAB_STENCIL_LDS && tile_divides(a.g, L, 1);
    const size_t lds = use_lds ? (size_t)2 * 3 * (L.block.x + 2) * (L.block.y + 2) * sizeof(T) : 0;
    if (rec) {
        record_launch(rec, kind_code(KK_MOM, mode | (use_lds ? STAGE_LDS : 0), sizeof(T) == 4), L.grid, L.block, lds, b);
        return hipSuccess;
    }
    if (use_lds) launch_mom_modes<T, true>(mode, b, L, lds, s);
    else launch_mom_modes<T, false>(mode, b, L, 0, s);
    return hipGetLastError();
}

bool mom_pair_supported(const Grid& g, const StencilLaunch& L) {
    const int bx = (int)L.block.x, by = (int)L.block.y;
    // at most two halo cells of V per thread (4 (BX + 2) + 4 BY of them) and
    // one ring cell per thread (2 BX + 2 BY of them)
    return bx == 64 && by == DNSLAB_PROWS && g.nx % bx == 0 && g.ny % by == 0 && 4 * (bx + 2) + 4 * by <= 2 * bx * by &&
           2 * (bx + by) <= bx * by;
}

template <typename T>
hipError_t launch_mom_pair(int pair, const MomPairArgs<T>& a, const StencilLaunch& L, hipStream_t s, Recorder* rec) {
    if (!mom_pair_supported(a.g, L) || (pair != 0 && pair != 1)) return hipErrorInvalidValue;
    MomPairArgs<T> b = a;
    b.kc = L.kc;
    const size_t lds = (size_t)6 * ((L.block.x + 4) * (L.block.y + 4) + (L.block.x + 2) * (L.block.y + 2)) * sizeof(T);
    if (rec) {
        record_launch(rec, kind_code(KK_MOMPAIR, pair, sizeof(T) == 4), L.grid, L.block, lds, b);
        return hipSuccess;
    }
    if (pair == 0) hipLaunchKernelGGL((k_mom_pair<T, 0>), L.grid, L.block, lds, s, b);
    else hipLaunchKernelGGL((k_mom_pair<T, 1>), L.grid, L.block, lds, s, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sca_pair(int pair, const ScaPairArgs<T>& a, const StencilLaunch& L, hipStream_t s, Recorder* rec) {
    if (!mom_pair_supported(a.g, L) || (pair != 0 && pair != 1)) return hipErrorInvalidValue;
    ScaPairArgs<T> b = a;
    b.kc = L.kc;
    const size_t tv = (size_t)(L.block.x + 4) * (L.block.y + 4), tw = (size_t)(L.block.x + 2) * (L.block.y + 2);
    const size_t lds = (6 * tv + 2 * tw) * sizeof(T) + 2 * tv;
    if (rec) {
        record_launch(rec, kind_code(KK_SCAPAIR, pair, sizeof(T) == 4), L.grid, L.block, lds, b);
        return hipSuccess;
    }
    if (pair == 0) hipLaunchKernelGGL((k_sca_pair<T, 0>), L.grid, L.block, lds, s, b);
    else hipLaunchKernelGGL((k_sca_pair<T, 1>), L.grid, L.block, lds, s, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sca_stage(int mode, const ScaArgs<T>& a, const StencilLaunch& L, hipStream_t s, Recorder* rec) {
    ScaArgs<T> b = a;
    b.kc = L.kc;
    if (rec) {
        record_launch(rec, kind_code(KK_SCA, mode, sizeof(T) == 4), L.grid, L.block, 0, b);
        return hipSuccess;
    }
    switch (mode) {
        case ST_FIRST: hipLaunchKernelGGL((k_sca_stage<T, ST_FIRST>), L.grid, L.block, 0, s, b); break;
        case ST_HALF: hipLaunchKernelGGL((k_sca_stage<T, ST_HALF>), L.grid, L.block, 0, s, b); break;
        case ST_FULL: hipLaunchKernelGGL((k_sca_stage<T, ST_FULL>), L.grid, L.block, 0, s, b); break;
        case ST_LAST: hipLaunchKernelGGL((k_sca_stage<T, ST_LAST>), L.grid, L.block, 0, s, b); break;
        default: hipLaunchKernelGGL((k_sca_stage<T, ST_RHS>), L.grid, L.block, 0, s, b); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_filter(const FiltArgs<T>& a, const StencilLaunch& L, hipStream_t s, Recorder* rec) {
    FiltArgs<T> b = a;
    b.kc = L.kc;
    // the LDS-tiled variant when the tile divides the grid in x and y; its
    // register-ring form for the 64 x DNSLAB_FROWS tile
    const bool use_lds = DNSLAB_FILTER_LDS && tile_divides(a.g, L, 3);
    const bool use_ring = use_lds && DNSLAB_FILTER_RING && L.block.x == 64 && L.block.y == DNSLAB_FROWS;
    const int nf = a.nf == 3 ? 3 : 1;
    const size_t lds = use_lds ? (size_t)2 * nf * (L.block.x + 6) * (L.block.y + 6) * sizeof(T) : 0;
    if (rec) {
        record_launch(rec, kind_code(KK_FILT, (a.nf == 3 ? 3 : 1) | (use_lds ? FILT_LDS : 0) | (use_ring ? FILT_RING : 0),
                                     sizeof(T) == 4), L.grid, L.block, lds, b);
        return hipSuccess;
    }
    if (use_ring) {
        if (a.nf == 3) hipLaunchKernelGGL((k_filter_ring<T, 3>), L.grid, L.block, lds, s, b);
        else hipLaunchKernelGGL((k_filter_ring<T, 1>), L.grid, L.block, lds, s, b);
    } else if (use_lds) {
        if (a.nf == 3) hipLaunchKernelGGL((k_filter_lds<T, 3>), L.grid, L.block, lds, s, b);
        else hipLaunchKernelGGL((k_filter_lds<T, 1>), L.grid, L.block, lds, s, b);
    } else {
        if (a.nf == 3) hipLaunchKernelGGL((k_filter<T, 3>), L.grid, L.block, 0, s, b);
        else hipLaunchKernelGGL((k_filter<T, 1>), L.grid, L.block, 0, s, b);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_correct(const CorrArgs<T>& a, const StencilLaunch& L, hipStream_t s, Recorder* rec) {
    CorrArgs<T> b = a;
    b.kc = L.kc;
    const bool ring = correct_ring_fits(a.g, L);
    const size_t lds = ring ? (size_t)2 * (L.block.x + 2) * (L.block.y + 2) * sizeof(T) : 0;
    if (rec) {
        record_launch(rec, kind_code(KK_CORR, ring ? 1 : 0, sizeof(T) == 4), L.grid, L.block, lds, b);
        return hipSuccess;
    }
    if (ring) hipLaunchKernelGGL((k_correct_ring<T>), L.grid, L.block, lds, s, b);
    else hipLaunchKernelGGL((k_correct<T>), L.grid, L.block, 0, s, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_div(const DivArgs<T>& a, const StencilLaunch& L, hipStream_t s, Recorder* rec) {
    DivArgs<T> b = a;
    b.kc = L.kc;
    if (rec) {
        record_launch(rec, kind_code(KK_DIV, 0, sizeof(T) == 4), L.grid, L.block, 0, b);
        return hipSuccess;
    }
    hipLaunchKernelGGL((k_div<T>), L.grid, L.block, 0, s, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rate(const T* u, const T* v, const T* w, const Grid& g, PartSoA part,
                       const StencilLaunch& L, hipStream_t s) {
    hipLaunchKernelGGL((k_rate<T>), L.grid, L.block, 0, s, u, v, w, g, L.kc, part);
    return hipGetLastError();
}

hipError_t launch_refine_res(const RefineResArgs& a, const StencilLaunch& L, hipStream_t s, Recorder* rec) {
    RefineResArgs b = a;
    b.kc = L.kc;
    const dim3 gib((unsigned)((a.ib.n + 255) / 256)), bib(256);
    if (rec) {
        record_launch(rec, kind_code(KK_REFRES, 0, 1), L.grid, L.block, 0, b);
        if (a.ib.n > 0) record_launch(rec, kind_code(KK_REFRES, 1, 1), gib, bib, 0, b);
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_refine_res, L.grid, L.block, 0, s, b);
    if (a.ib.n > 0) hipLaunchKernelGGL(k_refine_res_ib, gib, bib, 0, s, b);
    return hipGetLastError();
}

hipError_t launch_refine_correct(const RefineCorrArgs& a, const StencilLaunch& L, hipStream_t s, Recorder* rec) {
    RefineCorrArgs b = a;
    b.kc = L.kc;
    const bool ring = correct_ring_fits(a.g, L);
    const size_t lds = ring ? (size_t)2 * (L.block.x + 2) * (L.block.y + 2) * sizeof(double) : 0;
    if (rec) {
        record_launch(rec, kind_code(KK_REFCORR, ring ? 1 : 0, 1), L.grid, L.block, lds, b);
        return hipSuccess;
    }
    if (ring) hipLaunchKernelGGL(k_refine_correct_ring, L.grid, L.block, lds, s, b);
    else hipLaunchKernelGGL(k_refine_correct, L.grid, L.block, 0, s, b);
    return hipGetLastError();
}

hipError_t launch_advance(const AdvanceArgs& a, hipStream_t s, Recorder* rec) {
    if (rec) {
        record_launch(rec, kind_code(KK_ADVANCE, 0, 0), dim3(1), dim3(1024), 0, a);
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_diag(const DiagArgs& a, hipStream_t s, Recorder* rec) {
    if (rec) {
        record_launch(rec, kind_code(KK_DIAG, 0, 0), dim3(1), dim3(1024), 0, a);
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_diag, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

namespace {
template <typename T>
hipError_t batched_typed(int base, int mode, const void* tab, const unsigned* st, int ns, unsigned nb, dim3 blk,
                         size_t lds, hipStream_t s) {
    const dim3 grid(nb);
    switch (base) {
        case KK_MOM: {
            auto t = (const BRec<MomArgs<T>>*)tab;
            if (mode & STAGE_LDS) {
                switch (mode & 7) {
                    case ST_FIRST: hipLaunchKernelGGL((k_mom_stage_b<T, ST_FIRST, true>), grid, blk, lds, s, t, st, ns); break;
                    case ST_HALF: hipLaunchKernelGGL((k_mom_stage_b<T, ST_HALF, true>), grid, blk, lds, s, t, st, ns); break;
                    case ST_FULL: hipLaunchKernelGGL((k_mom_stage_b<T, ST_FULL, true>), grid, blk, lds, s, t, st, ns); break;
                    case ST_LAST: hipLaunchKernelGGL((k_mom_stage_b<T, ST_LAST, true>), grid, blk, lds, s, t, st, ns); break;
                    default: hipLaunchKernelGGL((k_mom_stage_b<T, ST_RHS, true>), grid, blk, lds, s, t, st, ns); break;
                }
            } else {
                switch (mode & 7) {
                    case ST_FIRST: hipLaunchKernelGGL((k_mom_stage_b<T, ST_FIRST, false>), grid, blk, 0, s, t, st, ns); break;
                    case ST_HALF: hipLaunchKernelGGL((k_mom_stage_b<T, ST_HALF, false>), grid, blk, 0, s, t, st, ns); break;
                    case ST_FULL: hipLaunchKernelGGL((k_mom_stage_b<T, ST_FULL, false>), grid, blk, 0, s, t, st, ns); break;
                    case ST_LAST: hipLaunchKernelGGL((k_mom_stage_b<T, ST_LAST, false>), grid, blk, 0, s, t, st, ns); break;
                    default: hipLaunchKernelGGL((k_mom_stage_b<T, ST_RHS, false>), grid, blk, 0, s, t, st, ns); break;
                }
            }
            break;
        }
        case KK_MOMPAIR: {
            auto t = (const BRec<MomPairArgs<T>>*)tab;
            if (mode == 0) hipLaunchKernelGGL((k_mom_pair_b<T, 0>), grid, blk, lds, s, t, st, ns);
            else hipLaunchKernelGGL((k_mom_pair_b<T, 1>), grid, blk, lds, s, t, st, ns);
            break;
        }
        case KK_SCAPAIR: {
            auto t = (const BRec<ScaPairArgs<T>>*)tab;
            if (mode == 0) hipLaunchKernelGGL((k_sca_pair_b<T, 0>), grid, blk, lds, s, t, st, ns);
            else hipLaunchKernelGGL((k_sca_pair_b<T, 1>), grid, blk, lds, s, t, st, ns);
            break;
        }
        case KK_SCA: {
            auto t = (const BRec<ScaArgs<T>>*)tab;
            switch (mode) {
                case ST_FIRST: hipLaunchKernelGGL((k_sca_stage_b<T, ST_FIRST>), grid, blk, 0, s, t, st, ns); break;
                case ST_HALF: hipLaunchKernelGGL((k_sca_stage_b<T, ST_HALF>), grid, blk, 0, s, t, st, ns); break;
                case ST_FULL: hipLaunchKernelGGL((k_sca_stage_b<T, ST_FULL>), grid, blk, 0, s, t, st, ns); break;
                case ST_LAST: hipLaunchKernelGGL((k_sca_stage_b<T, ST_LAST>), grid, blk, 0, s, t, st, ns); break;
                default: hipLaunchKernelGGL((k_sca_stage_b<T, ST_RHS>), grid, blk, 0, s, t, st, ns); break;
            }
            break;
        }
        case KK_FILT: {
            auto t = (const BRec<FiltArgs<T>>*)tab;
            const bool three = (mode & 7) == 3;
            if (mode & FILT_RING) {
                if (three) hipLaunchKernelGGL((k_filter_ring_b<T, 3>), grid, blk, lds, s, t, st, ns);
                else hipLaunchKernelGGL((k_filter_ring_b<T, 1>), grid, blk, lds, s, t, st, ns);
            } else if (mode & FILT_LDS) {
                if (three) hipLaunchKernelGGL((k_filter_lds_b<T, 3>), grid, blk, lds, s, t, st, ns);
                else hipLaunchKernelGGL((k_filter_lds_b<T, 1>), grid, blk, lds, s, t, st, ns);
            } else {
                if (three) hipLaunchKernelGGL((k_filter_b<T, 3>), grid, blk, 0, s, t, st, ns);
                else hipLaunchKernelGGL((k_filter_b<T, 1>), grid, blk, 0, s, t, st, ns);
            }
            break;
        }
        case KK_CORR:
            if (mode == 1)
                hipLaunchKernelGGL((k_correct_ring_b<T>), grid, blk, lds, s, (const BRec<CorrArgs<T>>*)tab, st, ns);
            else
                hipLaunchKernelGGL((k_correct_b<T>), grid, blk, 0, s, (const BRec<CorrArgs<T>>*)tab, st, ns);
            break;
        case KK_DIV:
            hipLaunchKernelGGL((k_div_b<T>), grid, blk, 0, s, (const BRec<DivArgs<T>>*)tab, st, ns);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_batched_stencil(int kind, const void* tab, const unsigned* st, int ns, unsigned nb, dim3 blk,
                                  size_t lds, hipStream_t s) {
    const int base = kind >> 8, mode = (kind >> 1) & 127, fp32 = kind & 1;
    if (base == KK_REFRES) {
        if (mode == 1) hipLaunchKernelGGL(k_refine_res_ib_b, dim3(nb), blk, 0, s, (const BRec<RefineResArgs>*)tab, st, ns);
        else hipLaunchKernelGGL(k_refine_res_b, dim3(nb), blk, 0, s, (const BRec<RefineResArgs>*)tab, st, ns);
        return hipGetLastError();
    }
    if (base == KK_REFCORR) {
        if (mode == 1)
            hipLaunchKernelGGL(k_refine_correct_ring_b, dim3(nb), blk, lds, s, (const BRec<RefineCorrArgs>*)tab, st, ns);
        else
            hipLaunchKernelGGL(k_refine_correct_b, dim3(nb), blk, 0, s, (const BRec<RefineCorrArgs>*)tab, st, ns);
        return hipGetLastError();
    }
    if (base == KK_ADVANCE) {
        hipLaunchKernelGGL(k_advance_b, dim3(nb), blk, 0, s, (const BRec<AdvanceArgs>*)tab, st, ns);
        return hipGetLastError();
    }
    if (base == KK_DIAG) {
        hipLaunchKernelGGL(k_diag_b, dim3(nb), blk, 0, s, (const BRec<DiagArgs>*)tab, st, ns);
        return hipGetLastError();
    }
    return fp32 ? batched_typed<float>(base, mode, tab, st, ns, nb, blk, lds, s)
                : batched_typed<double>(base, mode, tab, st, ns, nb, blk, lds, s);
}

hipError_t launch_set_rate(PartSoA part, int np, StepScalars* sc, hipStream_t s) {
    hipLaunchKernelGGL(k_set_rate, dim3(1), dim3(1024), 0, s, part, np, sc);
    return hipGetLastError();
}

#define DNSLAB_INST(T)                                                                                              \
    template hipError_t launch_mom_stage<T>(int, const MomArgs<T>&, const StencilLaunch&, hipStream_t, Recorder*); \
    template hipError_t launch_mom_pair<T>(int, const MomPairArgs<T>&, const StencilLaunch&, hipStream_t, Recorder*); \
    template hipError_t launch_sca_stage<T>(int, const ScaArgs<T>&, const StencilLaunch&, hipStream_t, Recorder*); \
    template hipError_t launch_sca_pair<T>(int, const ScaPairArgs<T>&, const StencilLaunch&, hipStream_t, Recorder*); \
    template hipError_t launch_filter<T>(const FiltArgs<T>&, const StencilLaunch&, hipStream_t, Recorder*);        \
    template hipError_t launch_correct<T>(const CorrArgs<T>&, const StencilLaunch&, hipStream_t, Recorder*);       \
    template hipError_t launch_div<T>(const DivArgs<T>&, const StencilLaunch&, hipStream_t, Recorder*);            \
    template hipError_t launch_rate<T>(const T*, const T*, const T*, const Grid&, PartSoA,                        \
                                       const StencilLaunch&, hipStream_t);
DNSLAB_INST(double)
DNSLAB_INST(float)
#undef DNSLAB_INST

}  // namespace dnslab
