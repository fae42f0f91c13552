// C ABI of libdnslab: context management and the sequencing of one
// projection time step (Sections 2.1, 2.2 and 2.4 of arXiv 2204.02107).
// Host code only; every arithmetic step runs in the kernels of stencil.hip
// and fft.hip, enqueued on the caller's stream.
#include "dnslab.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "fft.h"
#include "particles.h"
#include "postproc.h"
#include "stencil.h"

using namespace dnslab;

namespace {

thread_local std::string g_thread_err;
constexpr int RING_CAP = 4096;
constexpr int PROF_POOL = 32768;

enum KernelId { K_NONE = -1, K_MOM = 0, K_SCA, K_FXF, K_FY, K_FZ, K_FXI, K_FILT, K_FILTC, K_CORR, K_DIV, K_IB,
                K_ADV, K_DIAG, K_REF, K_PART, K_FYZ, K_MOMP, K_SCAP, K_COUNT };
const char* const kKernelNames[K_COUNT] = {"mom_stage", "scalar_stage", "fft_x_fwd", "fft_y", "fft_z", "fft_x_inv",
                                            "filter", "filter_c", "correct", "div", "ib_rhs", "advance", "diag",
                                            "refine_res", "particles", "fft_yz", "mom_pair", "scalar_pair"};

bool is_2a3b(int n) {
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}
int pow2_floor(long long v) {
    int p = 1;
    while ((long long)p * 2 <= v) p *= 2;
    return p;
}
int ilog2(int v) {
    int l = 0;
    while ((1 << (l + 1)) <= v) ++l;
    return l;
}
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Device memory of a context or pool: the caller's allocator when one is
// given (e.g. PyTorch's caching allocator), else hipMalloc / hipFree.  Every
// block must be 256-byte aligned (the workspace layout relies on it).
struct DevAlloc {
    void* (*alloc)(size_t, void*) = nullptr;
    void (*free_)(void*, void*) = nullptr;
    void* user = nullptr;
};

void* dev_alloc(const DevAlloc& a, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    void* p = nullptr;
    if (a.alloc) {
        p = a.alloc(bytes, a.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (p && (reinterpret_cast<uintptr_t>(p) & 255u) != 0) {
        // unusable: the kernels' vector loads and the layout need 256-byte alignment
        if (a.free_) a.free_(p, a.user);
        else (void)hipFree(p);
        p = nullptr;
    }
    return p;
}

void dev_free(const DevAlloc& a, void* p) {
    if (!p) return;
    if (a.free_) a.free_(p, a.user);
    else (void)hipFree(p);
}

DevAlloc alloc_of(const dnslab_params* P) {
    DevAlloc a;
    a.alloc = P->alloc;
    a.free_ = P->free_;
    a.user = P->alloc_user;
    return a;
}

struct Layout {
    size_t esz;           // field element size
    long long n;
    int m, sx;            // fft
    int nl_x, ls_x, lg_tx_y, lg_tx_z;
    int xtw_lds;          // x passes stage their twiddle tables in LDS
    int yz, lg_ca, lg_cb;  // fused plane pass (plane-major spectrum) and its LDS chunks
    AxisPlan px, py, pz;
    StencilLaunch L;       // momentum and scalar stage kernels
    StencilLaunch L1;      // one-cell-per-thread kernels (div, refinement residual, rate)
    StencilLaunch LC;      // the velocity correction (64 x DNSLAB_FROWS tiles: its register-ring form)
    StencilLaunch LF;      // filter
    StencilLaunch LP;      // fused RK4 stage pairs
    int nparts;            // partial-result slots (max block count of the reducing kernels)
    int nfields;           // work fields: 13, plus 3 for the projected velocity when the filter is on
    // byte offsets inside the workspace
    size_t off_flags, off_fields, off_spec, off_tw, off_s2, off_forced, off_part, off_sc, off_ring;
    size_t total;
    int nforced_cap;
};

int validate(const dnslab_params* P, std::string& why) {
    if (!P) { why = "params is NULL"; return DNSLAB_EINVAL; }
    if (P->precision != DNSLAB_FP64 && P->precision != DNSLAB_FP32_REFINE) { why = "bad precision"; return DNSLAB_EINVAL; }
    // FFT lines are staged whole in LDS (160 KB per CU on gfx950): lengths up
    // to 4096 (FP64) / 8192 (FP32) along x (a half-length complex line, its
    // twiddles and the real-transform twist: 98 KB at the limit) and 2048 /
    // 4096 along y and z (a column and its twiddles: 64 KB).
    const int fp64 = P->precision == DNSLAB_FP64;
    const int maxx = fp64 ? 4096 : 8192, maxyz = fp64 ? 2048 : 4096;
    if (P->nx < 4 || P->nx % 2 != 0 || !is_2a3b(P->nx) || P->nx > maxx) {
        why = "nx must be even, 2^a 3^b, 4 <= nx <= 4096 (FP64) / 8192 (FP32)";
        return DNSLAB_EUNSUPPORTED;
    }
    for (int n : {P->ny, P->nz})
        if (!is_2a3b(n) || n > maxyz) { why = "ny, nz must be 1 or 2^a 3^b <= 2048 (FP64) / 4096 (FP32)"; return DNSLAB_EUNSUPPORTED; }
    const long long n = (long long)P->nx * P->ny * P->nz;
    if (n >= (1LL << 31)) { why = "grid too large (>= 2^31 cells)"; return DNSLAB_EUNSUPPORTED; }
    if (!(P->lx > 0 && P->ly > 0 && P->lz > 0)) { why = "box lengths must be positive"; return DNSLAB_EINVAL; }
    if (!(P->tau_f > 0)) { why = "tau_f must be positive"; return DNSLAB_EINVAL; }
    if (P->n_piter < 0 || P->n_piter > 64) { why = "n_piter out of range"; return DNSLAB_EINVAL; }
    if (P->project_each_stage != 0 && P->project_each_stage != 1) { why = "project_each_stage must be 0 or 1"; return DNSLAB_EINVAL; }
    if ((P->alloc == nullptr) != (P->free_ == nullptr)) { why = "alloc and free_ must both be set or both be NULL"; return DNSLAB_EINVAL; }
    if (!(P->dt_fixed > 0)) {
        if (!(P->cfl > 0) || !(P->u_ref > 0)) { why = "adaptive dt needs cfl > 0 and u_ref > 0"; return DNSLAB_EINVAL; }
    }
    if (!std::isfinite(P->nu) || !std::isfinite(P->alpha_c) || !std::isfinite(P->body[0]) ||
        !std::isfinite(P->body[1]) || !std::isfinite(P->body[2])) {
        why = "non-finite parameter";
        return DNSLAB_EINVAL;
    }
    return DNSLAB_OK;
}

Grid make_grid(const dnslab_params* P) {
    Grid g;
    g.nx = P->nx; g.ny = P->ny; g.nz = P->nz;
    g.nxy = (long long)P->nx * P->ny;
    g.n = g.nxy * P->nz;
    g.d[0] = P->lx / P->nx; g.d[1] = P->ly / P->ny; g.d[2] = P->lz / P->nz;
    for (int a = 0; a < 3; ++a) {
        g.inv2d[a] = 1.0 / (2.0 * g.d[a]);
        g.inv4d[a] = 1.0 / (4.0 * g.d[a]);
        g.invd2[a] = 1.0 / (g.d[a] * g.d[a]);
    }
    g.dv = g.d[0] * g.d[1] * g.d[2];
    return g;
}

#ifndef DNSLAB_ROWS
#define DNSLAB_ROWS 4          // block height of the radius-1 stencil kernels
#endif
#ifndef DNSLAB_KC
#define DNSLAB_KC 0            // z cells per thread (0: from the grid size)
#endif
#ifndef DNSLAB_FKC
#define DNSLAB_FKC 0
#endif
#ifndef DNSLAB_XLS_MOD
#define DNSLAB_XLS_MOD 2       // x-pass LDS line stride modulo 16 (make_layout)
#endif
// Least z cells per thread of the filter (and of the velocity correction,
// which shares its launch): the radius-3 filter
// re-reads 6 halo planes per chunk.  24 in both forms since the filter runs
// as a register-ring march (512x256x192: filter 345 -> 305 us FP64,
// 191 -> 172 us FP32; 1024x512x256 already has 32).
#ifndef DNSLAB_FKC_MIN
#define DNSLAB_FKC_MIN 24
#endif
#ifndef DNSLAB_FKC_MIN32
#define DNSLAB_FKC_MIN32 24
#endif
// below this many blocks of 64 x DNSLAB_FROWS tiles, the filter and the
// correction take 64 x 8 tiles with the shorter chunks below
#ifndef DNSLAB_RING_MIN_BLOCKS
#define DNSLAB_RING_MIN_BLOCKS 1024
#endif
// Longer filter chunks where the 64 x DNSLAB_FROWS tiles still give this
// many blocks.
#ifndef DNSLAB_FKC_LONG
#define DNSLAB_FKC_LONG 64
#endif
#ifndef DNSLAB_FKC_LONG_BLOCKS
#define DNSLAB_FKC_LONG_BLOCKS 2048
#endif
#ifndef DNSLAB_FKC_MIN_SMALL
#define DNSLAB_FKC_MIN_SMALL 12
#endif
#ifndef DNSLAB_FKC_MIN_SMALL32
#define DNSLAB_FKC_MIN_SMALL32 8
#endif
// FFT passes: x lines per block grow while the block stays within these
// threads and LDS bytes; y/z column tiles within this much LDS.
#ifndef DNSLAB_XPASS_THREADS
#define DNSLAB_XPASS_THREADS 256
#endif
#ifndef DNSLAB_COL_PIPE
// Pipelined column passes (asynchronous LDS loads, several tiles per block)
// by tile count when set; off by default: measured slower than one tile per
// block on 1024x512x256 (y 433 -> 442, z 552 -> 594 us FP64) and on
// 512x256x192 (z 107 -> 146 us), where the plain pass keeps 2-4 blocks per CU
// against the pipeline's 1-2 (two tile buffers per block)
#define DNSLAB_COL_PIPE 0
#endif
#ifndef DNSLAB_XPASS_TW_LDS_MAX_M
// x passes stage their W_m and twist tables in LDS up to this half length m
// and read them through the caches beyond: on 1024x512x256 (m = 512) the
// tables took half of each block's LDS and reading them through the caches
// took the passes from 552 / 712 to 406 / 496 us (FP64 forward / inverse);
// on 256x128x96 (m = 128) staging them stays 5-7% faster
#define DNSLAB_XPASS_TW_LDS_MAX_M 256
#endif
#ifndef DNSLAB_XPASS_LDS_KB
#define DNSLAB_XPASS_LDS_KB 48
#endif
#ifndef DNSLAB_YZ
#define DNSLAB_YZ 1            // fused y/z pass when a (ky, kz) plane fits one block
#endif
#ifndef DNSLAB_YZ_LDS_KB
#define DNSLAB_YZ_LDS_KB 160
#endif
#ifndef DNSLAB_YZ_MAX_PLANE
#define DNSLAB_YZ_MAX_PLANE 8192   // largest ny * nz given to the fused pass (FP64)
#endif
#ifndef DNSLAB_YZ_MAX_PLANE32
#define DNSLAB_YZ_MAX_PLANE32 16384   // the same for the FP32 form (1024-thread blocks)
#endif
#ifndef DNSLAB_FORK_EARLY_CELLS
#define DNSLAB_FORK_EARLY_CELLS (1LL << 23)   // FP64: from this grid size the scalar half forks before the momentum stages
#endif
#ifndef DNSLAB_SERIAL_CELLS64
#define DNSLAB_SERIAL_CELLS64 (1LL << 26)     // FP64: from this grid size a step runs on one stream
#endif
#ifndef DNSLAB_FORK_EARLY_CELLS32
#define DNSLAB_FORK_EARLY_CELLS32 (1LL << 23)   // the same for the FP32 form
#endif
#ifndef DNSLAB_OVERLAP
#define DNSLAB_OVERLAP 1       // run the scalar half of a step on a second stream
#endif
#ifndef DNSLAB_COL_LDS_KB
#define DNSLAB_COL_LDS_KB 32
#endif
#ifndef DNSLAB_COL_FP32_WIDE
#define DNSLAB_COL_FP32_WIDE 0    // measured slower on 1024x512x256 (y 272 -> 288 us, z 382 -> 436 us)
#endif
#ifndef DNSLAB_PAIRS
#define DNSLAB_PAIRS 1         // RK4 stages two at a time (fused stage pairs) where the tile divides the grid
#endif
#ifndef DNSLAB_PAIR_MIN_BLOCKS64
#define DNSLAB_PAIR_MIN_BLOCKS64 256   // FP64 momentum pairs from this many blocks on (mom_pairs)
#endif
#ifndef DNSLAB_PAIR_MIN_KC
#define DNSLAB_PAIR_MIN_KC 16  // shortest z chunk for the scalar pairs and the FP32 momentum pairs
#endif
#ifndef DNSLAB_PKC_DIV
#define DNSLAB_PKC_DIV 1024    // stage-pair z chunk: nz * tiles per plane / this, clamped to [8, DNSLAB_PKC_MAX]
#endif
#ifndef DNSLAB_PKC_MAX
#define DNSLAB_PKC_MAX 32
#endif
// Longer stage-pair chunks where they still give this many blocks (the pair
// kernels re-read 4 halo planes and recompute 2 planes of the first stage per
// chunk).
#ifndef DNSLAB_PKC_LONG
#define DNSLAB_PKC_LONG 128
#endif
#ifndef DNSLAB_PKC_LONG_BLOCKS
#define DNSLAB_PKC_LONG_BLOCKS 2048
#endif
#ifndef DNSLAB_PKC_LONG32
#define DNSLAB_PKC_LONG32 64
#endif
#ifndef DNSLAB_PKC_LONG_BLOCKS32
#define DNSLAB_PKC_LONG_BLOCKS32 4096
#endif

// z chunk: enough blocks to fill the chip, each walking at least 4 planes.
int stencil_kc(const Grid& g, int rows, int forced) {
    if (forced > 0) return std::min(forced, g.nz);
    const StencilLaunch one = stencil_launch(g, rows, g.nz, 1);
    const long long cols = (long long)one.grid.x * one.grid.y;
    long long kc = (long long)g.nz * cols / 4096;
    kc = std::max(4LL, std::min(32LL, kc));
    return (int)std::min<long long>(kc, g.nz);
}

Layout make_layout(const dnslab_params* P, int n_forced) {
    Layout Lo = {};
    const Grid g = make_grid(P);
    Lo.esz = P->precision == DNSLAB_FP64 ? 8 : 4;
    const size_t csz = 2 * Lo.esz;
    Lo.n = g.n;
    Lo.m = P->nx / 2;
    Lo.sx = (int)align_up(Lo.m + 1, 16);
    Lo.px = make_axis_plan(Lo.m);
    Lo.py = make_axis_plan(P->ny);
    Lo.pz = make_axis_plan(P->nz);
    // x-pass line stride in LDS (complex values): the least stride >= m + 1
    // congruent to DNSLAB_XLS_MOD modulo 16 (-1: the least odd one).  The
    // Stockham passes give consecutive lanes consecutive lines, so the stride
    // sets which banks a wave's lanes hit; 2 (mod 16) measured best on
    // 1024x512x256 (x inverse 503 -> 491 us FP64, 331 -> 300 us FP32; 8 was
    // slower than odd)
    Lo.ls_x = ((Lo.m + 1) % 2 == 1) ? Lo.m + 1 : Lo.m + 2;
    if (DNSLAB_XLS_MOD >= 0) {
        Lo.ls_x = Lo.m + 1;
        while (Lo.ls_x % 16 != DNSLAB_XLS_MOD) ++Lo.ls_x;
    }
    Lo.xtw_lds = Lo.m < DNSLAB_XPASS_TW_LDS_MAX_M ? 1 : 0;
    const long long nlines = (long long)P->ny * P->nz;
    {
        int nl = 1;
        // (the LDS bounds count FP64 complex values in both precisions: the FP32
        // form keeps the FP64 tile shapes, hence as many blocks)
        while (nl * 2 * Lo.px.tpl <= DNSLAB_XPASS_THREADS &&
               ((size_t)nl * 2 * Lo.ls_x + (Lo.xtw_lds ? 2 * Lo.m + 1 : 0)) * 16 <= DNSLAB_XPASS_LDS_KB * 1024 &&
               nl < nlines)
            nl *= 2;
        Lo.nl_x = ilog2(nl);
    }
    auto pick_tx = [&](int n, const AxisPlan& ap, size_t lds_cap) {
        int tx = 1;
        const int cap = std::min(64, pow2_floor(2LL * (Lo.m + 1) - 1));
        while (tx * 2 <= cap && (size_t)tx * 2 * n * 16 <= lds_cap && tx * 2 * ap.tpl <= 1024) tx *= 2;
        return ilog2(tx);
    };
    Lo.lg_tx_y = pick_tx(P->ny, Lo.py, DNSLAB_COL_LDS_KB * 1024);
    // long y lines leave short row segments (at most 4 columns): twice the LDS
    // for the y pass (measured 10% faster on 1024x512x256; the z
    // pass, whose tiles are read with the larger row stride, is not)
    if ((1 << Lo.lg_tx_y) <= 4) Lo.lg_tx_y = pick_tx(P->ny, Lo.py, 2 * DNSLAB_COL_LDS_KB * 1024);
    Lo.lg_tx_z = pick_tx(P->nz, Lo.pz, DNSLAB_COL_LDS_KB * 1024);
    // FP32: twice the columns in the same LDS bytes, so that a tile's row
    // segments span as many bytes as in FP64 (with half-length segments the
    // L2 fetched whole lines twice: FETCH_SIZE twice the spectrum per pass)
    if (Lo.esz == 4 && DNSLAB_COL_FP32_WIDE) {
        auto widen = [&](int lg, int n, const AxisPlan& ap) {
            const int cap = std::min(64, pow2_floor(2LL * (Lo.m + 1) - 1));
            return (2 << lg) <= cap && (2LL << lg) * ap.tpl <= 1024 ? lg + 1 : lg;
        };
        Lo.lg_tx_y = widen(Lo.lg_tx_y, P->ny, Lo.py);
        Lo.lg_tx_z = widen(Lo.lg_tx_z, P->nz, Lo.pz);
    }
    // Fused plane pass: each of the nx/2 + 1 kx planes (ny * nz values) held
    // by one block in registers, its y and z lines transformed in LDS chunks.
    // It cuts two of the three column passes and their launches, but one
    // block per plane serialises a plane's work on one CU: measured 10%
    // faster steps for planes of 64 x 64, 3% slower for 96 x 64 and 8% for
    // 128 x 96 (FP64, 512-thread blocks), hence the plane-size limit; with
    // 1024-thread blocks (smaller planes, FP32) the pass gains 7-9% more.
    {
        const int nthr = yz_threads(P->ny, Lo.esz == 4);
        const long long max_plane = Lo.esz == 8 ? DNSLAB_YZ_MAX_PLANE : DNSLAB_YZ_MAX_PLANE32;
        if (DNSLAB_YZ && P->ny > 1 && P->nz > 1 && nthr > 0 && (long long)P->ny * P->nz <= max_plane &&
            yz_instance(Lo.esz == 4, nthr, (long long)P->ny * P->nz) >= 0 &&
            Lo.py.tpl <= nthr && Lo.pz.tpl <= nthr) {
            const size_t cap = (size_t)DNSLAB_YZ_LDS_KB * 1024;
            const size_t tw = (size_t)(P->ny + P->nz) * csz;
            auto lines = [&](int n, int other, const AxisPlan& ap) {
                int nl = 1;
                while (nl * 2 <= other && (long long)nl * 2 * ap.tpl <= nthr &&
                       tw + (size_t)n * (nl * 2 + 1) * csz <= cap)
                    nl *= 2;
                return tw + (size_t)n * (nl + 1) * csz <= cap ? nl : 0;
            };
            const int ca = lines(P->ny, P->nz, Lo.py), cb = lines(P->nz, P->ny, Lo.pz);
            if (ca > 0 && cb > 0) {
                Lo.yz = 1;
                Lo.lg_ca = ilog2(ca);
                Lo.lg_cb = ilog2(cb);
            }
        }
    }
    Lo.L = stencil_launch(g, DNSLAB_ROWS, stencil_kc(g, DNSLAB_ROWS, DNSLAB_KC), 1);
    Lo.L1 = Lo.L;
    // Filter and correction: 64 x DNSLAB_FROWS tiles with long z chunks (the
    // radius-3 filter re-reads 6 halo planes per chunk), their register-ring
    // forms, where that still gives DNSLAB_RING_MIN_BLOCKS blocks; on smaller
    // grids 64 x 8 tiles with shorter chunks, the LDS filter and the
    // one-cell-per-thread correction, which keep many more blocks (on
    // 192x96x64 the large tiles made the filter 28 -> 53 us and the
    // correction 12 -> 32 us: 24 blocks for 256 CUs).
    const int fkc_min = Lo.esz == 8 ? DNSLAB_FKC_MIN : DNSLAB_FKC_MIN32;
    Lo.LF = stencil_launch(g, DNSLAB_FROWS,
                           std::max(stencil_kc(g, DNSLAB_FROWS, DNSLAB_FKC), std::min(fkc_min, P->nz)), 1);
    const bool ring_geometry = Lo.LF.nblocks >= DNSLAB_RING_MIN_BLOCKS;
    if (ring_geometry && Lo.LF.kc < DNSLAB_FKC_LONG) {
        const StencilLaunch lf = stencil_launch(g, DNSLAB_FROWS, std::min(DNSLAB_FKC_LONG, P->nz), 1);
        if (lf.nblocks >= DNSLAB_FKC_LONG_BLOCKS) Lo.LF = lf;
    }
    if (!ring_geometry) {
        const int small_min = Lo.esz == 8 ? DNSLAB_FKC_MIN_SMALL : DNSLAB_FKC_MIN_SMALL32;
        Lo.LF = stencil_launch(g, 8, std::max(stencil_kc(g, 8, DNSLAB_FKC), std::min(small_min, P->nz)), 1);
    }
    {
        // the pair kernels read kc + 4 planes and evaluate their first stage on
        // kc + 2 planes per chunk: longer chunks than the single-stage kernels
        const StencilLaunch one = stencil_launch(g, DNSLAB_PROWS, g.nz, 1);
        const long long cols = (long long)one.grid.x * one.grid.y;
        const long long pkc = std::max(8LL, std::min((long long)DNSLAB_PKC_MAX, (long long)g.nz * cols / DNSLAB_PKC_DIV));
        Lo.LP = stencil_launch(g, DNSLAB_PROWS, (int)std::min<long long>(pkc, g.nz), 1);
        const int long_kc = Lo.esz == 8 ? DNSLAB_PKC_LONG : DNSLAB_PKC_LONG32;
        const int long_blocks = Lo.esz == 8 ? DNSLAB_PKC_LONG_BLOCKS : DNSLAB_PKC_LONG_BLOCKS32;
        if (Lo.LP.kc < long_kc) {
            const StencilLaunch lp = stencil_launch(g, DNSLAB_PROWS, std::min(long_kc, g.nz), 1);
            if (lp.nblocks >= long_blocks) Lo.LP = lp;
        }
    }
    Lo.LC = ring_geometry ? Lo.LF : Lo.L1;
    Lo.nparts = std::max(std::max(std::max(Lo.L.nblocks, Lo.L1.nblocks), Lo.LF.nblocks), Lo.LP.nblocks);
    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
    Lo.off_flags = take((size_t)g.n);
    Lo.nfields = P->filter ? 16 : 13;
    Lo.off_fields = take((size_t)Lo.nfields * g.n * Lo.esz);
    Lo.off_spec = take((size_t)Lo.sx * nlines * csz);
    Lo.off_tw = take((size_t)(Lo.m + P->ny + P->nz + Lo.m + 1) * csz);
    Lo.off_s2 = take((size_t)(Lo.m + 1 + P->ny + P->nz) * sizeof(double));
    Lo.nforced_cap = std::max(1, n_forced);
    Lo.off_forced = take((size_t)Lo.nforced_cap * (sizeof(long long) + 5 * sizeof(double)));
    Lo.off_part = take((size_t)PF_COUNT * Lo.nparts * sizeof(double));
    Lo.off_sc = take(sizeof(StepScalars));
    Lo.off_ring = take((size_t)RING_CAP * sizeof(DiagRec));
    Lo.total = off;
    return Lo;
}

// exp(-2 pi i j / n) in long double, rounded once.
void twiddles(int n, std::vector<long double>& re, std::vector<long double>& im, int count) {
    re.resize(count);
    im.resize(count);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int j = 0; j < count; ++j) {
        const long double ang = -2.0L * pi * (long double)j / (long double)n;
        re[j] = cosl(ang);
        im[j] = sinl(ang);
    }
}

// sin^2(2 pi m / n) / h^2 with exact zeros where 2m is a multiple of n.
void sin2_table(int n, int count, double h, double* out) {
    for (int m = 0; m < count; ++m) {
        if ((2LL * m) % n == 0) { out[m] = 0.0; continue; }
        const double s = std::sin(2.0 * M_PI * m / n);
        out[m] = s * s / (h * h);
    }
}

}  // namespace

struct dnslab_ctx {
    dnslab_params P;
    DevAlloc da;           // device memory: the caller's allocator or hipMalloc
    hipStream_t stream;
    Grid g;
    Layout Lo;
    void* ws;
    void *u, *v, *w, *p, *c;
    uint8_t* flags;
    void* f[16];           // A0..2, B0..2, Cb0..2, R0, CA, CS1, CS2, V0..2 (filter on)
    void* spec;
    void *wx, *wy, *wz, *tw;
    double *sx2, *sy2, *sz2;
    long long* fidx;
    double *fS, *fuset, *fcset;
    int nforced;
    PartSoA part;
    StepScalars* sc;
    DiagRec* ring;
    bool any_solid;
    void* ib_buf;          // near-solid list: idx (int), mask (uint8), saved r0 (field type)
    void* ib_r0;
    IBList ib;
    bool rate_valid;
    long long host_step;
    unsigned long long* hist_dev;   // histogram counters (allocated on first use)
    unsigned long long* hist_host;
    void* psort_buf;       // particle-sort scratch (allocated on first use, grown as needed)
    size_t psort_bytes;    // its size
    DiagRec* pinned;       // host staging for diagnostics
    StepScalars* pinned_sc;
    std::string err;
    Recorder* rec;         // non-NULL: launches are recorded for batched replay, not issued
    hipStream_t cur;       // stream of the launches being enqueued (stream, or aux for the scalar work)
    // The scalar transport of step n only needs the projected velocity of
    // step n; it runs on a second stream, overlapping the pressure solves of
    // step n + 1 (see one_step).
    bool overlap;          // defer the scalar work to aux (plain contexts; not when recording)
    int pairs_mode = -1;   // RK4 stage pairs: -1 by grid size, 0 never, 1 wherever the tile divides the grid
    int fft_pipe_mode = -1;   // pipelined column passes: -1 by tile count, 0 never, 1 wherever they apply
    hipStream_t aux;       // created on first use
    hipEvent_t ev_fork, ev_join;
    bool tail_pending;     // scalar work of the last step taken not yet enqueued
    bool join_pending;     // stream has not yet waited for the last enqueued scalar work
    // graph replay of whole steps
    int graph_steps;       // k steps per graph (0: launch by launch)
    hipGraphExec_t gexec;
    int gexec_steps;
    // profiling
    int prof_kid;
    std::vector<hipEvent_t> ev;
    int ev_used;
    double prof_ms;
    long long prof_n;
};

namespace {

int fail(dnslab_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    else g_thread_err = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, DNSLAB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int prof_flush(dnslab_ctx* x) {
    if (x->ev_used == 0) return DNSLAB_OK;
    HIPCHK(x, hipStreamSynchronize(x->stream));
    if (x->aux) HIPCHK(x, hipStreamSynchronize(x->aux));
    for (int i = 0; i + 1 < x->ev_used; i += 2) {
        float ms = 0;
        HIPCHK(x, hipEventElapsedTime(&ms, x->ev[i], x->ev[i + 1]));
        x->prof_ms += ms;
        x->prof_n += 1;
    }
    x->ev_used = 0;
    return DNSLAB_OK;
}

// Bracket a launch with events when that kernel is being profiled.
struct Prof {
    dnslab_ctx* x;
    bool on;
    Prof(dnslab_ctx* x_, int kid) : x(x_), on(x_->prof_kid == kid && !x_->rec) {
        if (on) {
            if (x->ev_used + 2 > (int)x->ev.size()) prof_flush(x);
            (void)hipEventRecord(x->ev[x->ev_used], x->cur);
        }
    }
    ~Prof() {
        if (on) {
            (void)hipEventRecord(x->ev[x->ev_used + 1], x->cur);
            x->ev_used += 2;
        }
    }
};

#define LAUNCH(ctx, kid, expr)                                                             \
    do {                                                                                   \
        hipError_t e_;                                                                     \
        {                                                                                  \
            Prof pr_(ctx, kid);                                                            \
            e_ = (expr);                                                                   \
        }                                                                                  \
        if (e_ != hipSuccess)                                                              \
            return fail(ctx, DNSLAB_EHIP, std::string("launch: ") + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
Forcing forcing_of(dnslab_ctx* x) {
    Forcing f;
    f.idx = x->fidx;
    f.S = x->fS;
    f.uset = x->fuset;
    f.cset = x->fcset;
    f.n = x->nforced;
    f.inv_tau = 1.0 / x->P.tau_f;
    return f;
}

// The FFT description of a grid whose spectrum starts at spec, its twiddle
// tables at w (W_m, W_ny, W_nz, then e^{-2 pi i k/nx} for k <= m) and its
// symbol tables at s2 (x, y, z).
template <typename T>
FFTArgs<T> fft_args_of(const Layout& Lo, const Grid& g, void* spec, const void* w, const double* s2) {
    FFTArgs<T> a;
    a.g = g;
    a.m = Lo.m;
    a.sx = Lo.sx;
    a.ps = Lo.yz ? g.ny * g.nz : 0;
    a.spec = (C2<T>*)spec;
    a.px = Lo.px;
    a.py = Lo.py;
    a.pz = Lo.pz;
    a.wx = (const C2<T>*)w;
    a.wy = a.wx + Lo.m;
    a.wz = a.wy + g.ny;
    a.tw = a.wz + g.nz;
    a.sx2 = s2;
    a.sy2 = s2 + Lo.m + 1;
    a.sz2 = a.sy2 + g.ny;
    a.inv_ntot = 1.0 / (double)g.n;
    a.xtw_lds = Lo.xtw_lds;
    a.col_pipe = DNSLAB_COL_PIPE ? -1 : 0;
    a.nl_x = Lo.nl_x;
    a.ls_x = Lo.ls_x;
    a.lg_tx_y = Lo.lg_tx_y;
    a.lg_tx_z = Lo.lg_tx_z;
    a.lg_ca = Lo.lg_ca;
    a.lg_cb = Lo.lg_cb;
    return a;
}

template <typename T>
FFTArgs<T> fft_args(dnslab_ctx* x) {
    FFTArgs<T> a = fft_args_of<T>(x->Lo, x->g, x->spec, x->wx, x->sx2);
    if (x->fft_pipe_mode != -1) a.col_pipe = x->fft_pipe_mode;
    return a;
}

// One FFT solve of Lap p = r (central-difference symbol, null modes zero).
template <typename T>
int poisson_solve(dnslab_ctx* x, const T* r, T* pout) {
    const FFTArgs<T> a = fft_args<T>(x);
    LAUNCH(x, K_FXF, launch_fft_x_fwd<T>(a, r, x->cur, x->rec));
    if (x->Lo.yz) {
        LAUNCH(x, K_FYZ, launch_fft_yz_solve<T>(a, x->cur, x->rec));
    } else {
        if (x->g.ny > 1) LAUNCH(x, K_FY, launch_fft_y<T>(a, false, x->cur, x->rec));
        LAUNCH(x, K_FZ, launch_fft_z_solve<T>(a, x->cur, x->rec));
        if (x->g.ny > 1) LAUNCH(x, K_FY, launch_fft_y<T>(a, true, x->cur, x->rec));
    }
    LAUNCH(x, K_FXI, launch_fft_x_inv<T>(a, pout, x->cur, x->rec));
    return DNSLAB_OK;
}

// Projection of Section 2.2 in three parts: r0 = div u* (project_div), the n
// IB iterations on the bound p (project_solve), and the velocity correction
// (project_correct).  In the FP32 form the last solve is refined once in FP64
// (iterative refinement): its residual r_n - Lap_h p_n is formed in FP64 from
// the FP32 fields, solved for a correction dp, and the velocity correction
// u = beta (u* - grad(p_n + dp)) is applied in FP64 arithmetic.
template <typename T>
int project_div(dnslab_ctx* x, const T* const us[3]) {
    DivArgs<T> d;
    for (int a = 0; a < 3; ++a) d.u[a] = us[a];
    d.out = (T*)x->f[9];
    d.g = x->g;
    LAUNCH(x, K_DIV, launch_div<T>(d, x->Lo.L1, x->cur, x->rec));
    return DNSLAB_OK;
}

// With no solid cell the IB iterates are identical: one solve gives them all.
int n_solves(const dnslab_ctx* x) { return x->any_solid ? x->P.n_piter : std::min(x->P.n_piter, 1); }
bool refining(const dnslab_ctx* x) { return x->P.precision == DNSLAB_FP32_REFINE && n_solves(x) > 0; }

// scr: three field-sized scratch arrays for the FP32 refinement (last iterate,
// residual, correction), which must not alias us; by default the B stage buffers.
template <typename T>
int project_solve(dnslab_ctx* x, const T* const us[3], void* const* scr = nullptr) {
    void* const* S = scr ? scr : x->f + 3;
    T* r0 = (T*)x->f[9];
    T* p = (T*)x->p;
    const int nit = n_solves(x);
    const bool refine = refining(x);
    T* p_last = refine ? (T*)S[0] : p;    // the last iterate goes to a scratch field when refining
    for (int it = 0; it < nit; ++it) {
        if (x->any_solid) LAUNCH(x, K_IB, launch_ib_rhs<T>(x->ib, x->g, p, r0, (T*)x->ib_r0, it == 0, x->cur, x->rec));
        int rc = poisson_solve<T>(x, r0, it == nit - 1 ? p_last : p);
        if (rc) return rc;
    }
    if constexpr (sizeof(T) == 4) {
        if (refine) {
            RefineResArgs ra;
            for (int a = 0; a < 3; ++a) ra.us[a] = (const float*)us[a];
            ra.p3 = (const float*)p;
            ra.p4 = (const float*)p_last;
            ra.flags = x->flags;
            ra.res = (float*)S[1];
            ra.g = x->g;
            ra.ib = x->ib;
            LAUNCH(x, K_REF, launch_refine_res(ra, x->Lo.L1, x->cur, x->rec));
            int rc = poisson_solve<float>(x, (const float*)S[1], (float*)S[2]);
            if (rc) return rc;
        }
    }
    return DNSLAB_OK;
}

template <typename T>
int project_correct(dnslab_ctx* x, const T* const us[3], T* const out[3], PartSoA part, void* const* scr = nullptr) {
    void* const* S = scr ? scr : x->f + 3;
    if constexpr (sizeof(T) == 4) {
        if (refining(x)) {
            RefineCorrArgs rc2;
            for (int a = 0; a < 3; ++a) { rc2.us[a] = (const float*)us[a]; rc2.out[a] = (float*)out[a]; }
            rc2.p4 = (const float*)S[0];
            rc2.dp = (const float*)S[2];
            rc2.p = (float*)x->p;
            rc2.flags = x->flags;
            rc2.g = x->g;
            rc2.part = part;
            LAUNCH(x, K_CORR, launch_refine_correct(rc2, x->Lo.LC, x->cur, x->rec));
            return DNSLAB_OK;
        }
    }
    CorrArgs<T> ca;
    for (int a = 0; a < 3; ++a) { ca.us[a] = us[a]; ca.out[a] = out[a]; }
    ca.p = (const T*)x->p;
    ca.flags = x->flags;
    ca.g = x->g;
    ca.part = part;
    LAUNCH(x, K_CORR, launch_correct<T>(ca, x->Lo.LC, x->cur, x->rec));
    return DNSLAB_OK;
}

template <typename T>
int project(dnslab_ctx* x, const T* const us[3], T* const out[3]) {
    int rc = project_div<T>(x, us);
    if (!rc) rc = project_solve<T>(x, us);
    if (!rc) rc = project_correct<T>(x, us, out, PartSoA{});
    return rc;
}

// RK4 stages two per pass where the pair kernels' tile divides the grid and
// the grid gives each block a z chunk long enough for the pipeline's four
// extra planes: measured, the momentum pairs gain on 256x128x96 in FP64
// (8-plane chunks: 261 -> 224 us per step) but lose in FP32 (139 -> 152 us),
// and the scalar pairs lose on it in both (152 -> 189, 104 -> 137 us), while
// on 1024x512x256 (32-plane chunks) both gain (FP64 momentum 12.0 -> 6.6 ms,
// scalar 7.6 -> 5.2 ms per step).
// dnslab_set_stage_pairs overrides the choice (pairs_mode 0: never, 1:
// wherever supported).
// FP64 momentum pairs on short z chunks pay only with a block per CU or more:
// with 8-plane chunks 64^3 (64 blocks) ran 1.11 Gcell-steps/s with single
// stages against 1.01 with pairs, 128x64x64 (128 blocks) 1.95 against 1.83,
// 192x96x64 (288) 3.00 either way, the 256x128x96 room (768) 3.80 against
// 3.95.
bool mom_pairs(const dnslab_ctx* x) {
    if (x->pairs_mode == 0 || !DNSLAB_PAIRS || !mom_pair_supported(x->g, x->Lo.LP)) return false;
    return x->pairs_mode == 1 || (x->Lo.esz == 8 && x->Lo.LP.nblocks >= DNSLAB_PAIR_MIN_BLOCKS64) ||
           x->Lo.LP.kc >= DNSLAB_PAIR_MIN_KC;
}
// The scalar's second pair reads c^n at the cells around its tile, so it
// cannot write c^n in place: the pairs run when the filter is on (the RK4
// result then goes to a work field).
bool sca_pairs(const dnslab_ctx* x) {
    if (x->pairs_mode == 0 || !DNSLAB_PAIRS || x->P.filter == 0 || !mom_pair_supported(x->g, x->Lo.LP)) return false;
    return x->pairs_mode == 1 || x->Lo.LP.kc >= DNSLAB_PAIR_MIN_KC;
}
// Partial-sum slots the scalar stages fill (divergence and, without the filter, CO2).
int sca_nblocks(const dnslab_ctx* x) { return sca_pairs(x) ? x->Lo.LP.nblocks : x->Lo.L.nblocks; }

template <typename T>
int scalar_rk4(dnslab_ctx* x, const T* const uvel[3], const double* dtp, double dt, T* cout, PartSoA pdiv,
               PartSoA psca) {
    T* C = (T*)x->c;
    T* CA = (T*)x->f[10];
    T* CS1 = (T*)x->f[11];
    T* CS2 = (T*)x->f[12];
    ScaArgs<T> s = {};
    for (int a = 0; a < 3; ++a) s.u[a] = uvel[a];
    s.flags = x->flags;
    s.dtp = dtp;
    s.dt = dt;
    s.frc = forcing_of<T>(x);
    s.alpha = x->P.alpha_c;
    s.g = x->g;
    s.acc = CA;
    const StencilLaunch& L = x->Lo.L;
    if (sca_pairs(x) && (const void*)cout != (const void*)C) {
        // two stages per pass: c^n -> acc after stage 2 (CA) and c2 (CS1);
        // then c2, c^n and acc -> c*
        ScaPairArgs<T> q = {};
        for (int a = 0; a < 3; ++a) q.u[a] = uvel[a];
        q.flags = s.flags;
        q.dtp = dtp;
        q.dt = dt;
        q.frc = s.frc;
        q.alpha = s.alpha;
        q.g = s.g;
        q.cin = C; q.acc = CA; q.out = CS1; q.part = pdiv;
        LAUNCH(x, K_SCAP, launch_sca_pair<T>(0, q, x->Lo.LP, x->cur, x->rec));
        q.cin = CS1; q.cn = C; q.accin = CA; q.acc = nullptr; q.out = cout; q.part = psca;
        LAUNCH(x, K_SCAP, launch_sca_pair<T>(1, q, x->Lo.LP, x->cur, x->rec));
        return DNSLAB_OK;
    }
    s.cs = C; s.out = CS1; s.part = pdiv;
    LAUNCH(x, K_SCA, launch_sca_stage<T>(ST_FIRST, s, L, x->cur, x->rec));
    s.cs = CS1; s.cn = C; s.out = CS2; s.part = PartSoA{};
    LAUNCH(x, K_SCA, launch_sca_stage<T>(ST_HALF, s, L, x->cur, x->rec));
    s.cs = CS2; s.cn = C; s.out = CS1;
    LAUNCH(x, K_SCA, launch_sca_stage<T>(ST_FULL, s, L, x->cur, x->rec));
    s.cs = CS1; s.cn = nullptr; s.out = cout; s.part = psca;
    LAUNCH(x, K_SCA, launch_sca_stage<T>(ST_LAST, s, L, x->cur, x->rec));
    return DNSLAB_OK;
}

template <typename T>
int ensure_rate(dnslab_ctx* x) {
    if (x->rate_valid || x->rec) return DNSLAB_OK;
    HIPCHK(x, launch_rate<T>((const T*)x->u, (const T*)x->v, (const T*)x->w, x->g, x->part, x->Lo.L1, x->stream));
    // launch_rate fills the rate partials of L1.nblocks blocks
    HIPCHK(x, launch_set_rate(x->part, x->Lo.L1.nblocks, x->sc, x->stream));
    x->rate_valid = true;
    return DNSLAB_OK;
}

// Projected velocity of the step just taken: the filter's input when the
// filter is on, else the velocity fields themselves.
template <typename T>
void projected_velocity(dnslab_ctx* x, T* V[3]) {
    const bool filt = x->P.filter != 0;
    for (int a = 0; a < 3; ++a) V[a] = filt ? (T*)x->f[13 + a] : (T*)(a == 0 ? x->u : a == 1 ? x->v : x->w);
}

// Scalar half of a step (Section 2.4: the CO2 is advanced after the projection
// with the projected velocity frozen): RK4 with the step's dt, the scalar's
// filter, and the step's diagnostics record.  Reads the projected velocity and
// the step scalars left by the velocity half; touches nothing else the
// velocity half of the next step uses.
template <typename T>
int scalar_half(dnslab_ctx* x) {
    const bool filt = x->P.filter != 0;
    T* V[3];
    projected_velocity<T>(x, V);
    const T* Vc[3] = {V[0], V[1], V[2]};
    T* C = (T*)x->c;
    T* CS2 = (T*)x->f[12];
    int rc = scalar_rk4<T>(x, Vc, &x->sc->last_dt, 0.0, filt ? CS2 : C, x->part, filt ? PartSoA{} : x->part);
    if (rc) return rc;
    if (filt) {
        FiltArgs<T> fa = {};
        fa.in[0] = CS2;
        fa.out[0] = C;
        fa.nf = 1;
        fa.flags = x->flags;
        fa.g = x->g;
        fa.part = x->part;
        LAUNCH(x, K_FILTC, launch_filter<T>(fa, x->Lo.LF, x->cur, x->rec));
    }
    DiagArgs d;
    d.part = x->part;
    d.np_vel = filt ? x->Lo.LF.nblocks : x->Lo.LC.nblocks;
    d.np_sca = filt ? x->Lo.LF.nblocks : sca_nblocks(x);
    d.np_div = sca_nblocks(x);
    d.sc = x->sc;
    d.ring = x->ring;
    d.ring_cap = RING_CAP;
    d.dv = x->g.dv;
    LAUNCH(x, K_DIAG, launch_diag(d, x->cur, x->rec));
    return DNSLAB_OK;
}

// Enqueue the deferred scalar half of the last step on the second stream,
// ordered after everything enqueued so far on the main stream.
template <typename T>
int flush_scalar_half(dnslab_ctx* x) {
    if (!x->tail_pending) return DNSLAB_OK;
    x->tail_pending = false;
    HIPCHK(x, hipEventRecord(x->ev_fork, x->stream));
    HIPCHK(x, hipStreamWaitEvent(x->aux, x->ev_fork, 0));
    x->cur = x->aux;
    const int rc = scalar_half<T>(x);
    x->cur = x->stream;
    if (rc) return rc;
    HIPCHK(x, hipEventRecord(x->ev_join, x->aux));
    x->join_pending = true;
    return DNSLAB_OK;
}

// Main stream waits for the scalar work enqueued on the second stream.
int join_scalar_half(dnslab_ctx* x) {
    if (!x->join_pending) return DNSLAB_OK;
    HIPCHK(x, hipStreamWaitEvent(x->stream, x->ev_join, 0));
    x->join_pending = false;
    return DNSLAB_OK;
}

int ensure_aux(dnslab_ctx* x) {
    if (x->aux) return DNSLAB_OK;
    HIPCHK(x, hipStreamCreateWithFlags(&x->aux, hipStreamNonBlocking));
    HIPCHK(x, hipEventCreateWithFlags(&x->ev_fork, hipEventDisableTiming));
    HIPCHK(x, hipEventCreateWithFlags(&x->ev_join, hipEventDisableTiming));
    return DNSLAB_OK;
}

// One time step (Sections 2.1, 2.2, 2.4).  Velocity half on the main stream:
// RK4 momentum to u*, div u*, the IB pressure iterations, the correction, the
// velocity filter and the step advance (t, step, next dt from the new Courant
// rate).  Scalar half: see scalar_half.  On a plain context the scalar half of
// step n is enqueued on the second stream once div u* of step n + 1 is
// enqueued (on large grids: before the momentum stages of step n + 1), so
// that it runs beside that step's work; the correction of step n + 1, which
// overwrites the projected velocity the scalar half reads, waits for it.
// When recording for the pool both halves go, in order, into one sequence.
template <typename T>
int one_step(dnslab_ctx* x) {
    int rc = ensure_rate<T>(x);
    if (rc) return rc;
    // (FP64 on the largest grids: one stream, see below)
    const bool defer = x->overlap && !x->rec && !(sizeof(T) == 8 && x->g.n >= DNSLAB_SERIAL_CELLS64);
    if (defer) {
        rc = ensure_aux(x);
        if (rc) return rc;
    }
    T* U[3] = {(T*)x->u, (T*)x->v, (T*)x->w};
    T* A[3] = {(T*)x->f[0], (T*)x->f[1], (T*)x->f[2]};
    T* B[3] = {(T*)x->f[3], (T*)x->f[4], (T*)x->f[5]};
    T* Cb[3] = {(T*)x->f[6], (T*)x->f[7], (T*)x->f[8]};
    const StencilLaunch& L = x->Lo.L;
    MomArgs<T> m = {};
    m.flags = x->flags;
    m.dtp = &x->sc->dt;
    m.frc = forcing_of<T>(x);
    m.nu = x->P.nu;
    for (int a = 0; a < 3; ++a) m.body[a] = x->P.body[a];
    m.g = x->g;
    // RK4 stages (Section 2.1), no pressure gradient.  In the per-stage
    // variant each stage value u_1, u_2, u_3 is projected in place (div, IB
    // iterations warm-started from the last pressure, correction) before the
    // next stage evaluates F on it; the accumulator sums the k's as usual.
    const bool per_stage = x->P.project_each_stage != 0;
    bool forked = false;
    // Where the scalar half of the last step forks: after div u* its work
    // overlaps the pressure solves only, whose passes leave the memory system
    // idle between their load and store phases (best when the solves are
    // long against the scalar half: the 256x128x96 room loses 7% forking
    // earlier).  On large grids the solves run closer to the bandwidth and
    // the scalar half outlasts them, stalling the correction that waits for
    // it, so there it forks before the momentum stages (FP32 512x256x192
    // +2.9%, 1024x512x256 +0.5%; FP64 512x256x192 5.53 -> 5.66
    // Gcell-steps/s).  On 1024x512x256 in FP64, where every kernel fills
    // the GPU many times over, one stream is faster still (5.84 forking
    // late, 5.69 early, 5.93 on one stream); in the FP32 form, whose scalar
    // pair leaves room on the CUs for the momentum pair beside it, two
    // streams stay faster (8.61 against 8.50).
    const long long fork_early = sizeof(T) == 8 ? DNSLAB_FORK_EARLY_CELLS : DNSLAB_FORK_EARLY_CELLS32;
    if (defer && x->g.n >= fork_early) {
        rc = flush_scalar_half<T>(x);
        if (rc) return rc;
        forked = true;
    }
    // the refinement scratch is the stage buffer not being projected
    auto project_stage = [&](T* const s[3], T* const other[3]) -> int {
        const T* const sc[3] = {s[0], s[1], s[2]};
        void* const scr[3] = {other[0], other[1], other[2]};
        int r = project_div<T>(x, sc);
        if (!r && defer && !forked) { r = flush_scalar_half<T>(x); forked = true; }
        if (!r) r = project_solve<T>(x, sc, scr);
        if (!r) r = project_correct<T>(x, sc, s, PartSoA{}, scr);
        return r;
    };
    if (!per_stage && mom_pairs(x)) {
        // two stages per pass: u^n -> acc after stage 2 (A) and u2 (B); then
        // u2, u^n and acc -> u* (Cb)
        MomPairArgs<T> q = {};
        q.flags = m.flags;
        q.dtp = m.dtp;
        q.frc = m.frc;
        q.nu = m.nu;
        for (int a = 0; a < 3; ++a) q.body[a] = m.body[a];
        q.g = m.g;
        for (int a = 0; a < 3; ++a) { q.vin[a] = U[a]; q.acc[a] = A[a]; q.out[a] = B[a]; }
        LAUNCH(x, K_MOMP, launch_mom_pair<T>(0, q, x->Lo.LP, x->cur, x->rec));
        for (int a = 0; a < 3; ++a) { q.vin[a] = B[a]; q.un[a] = U[a]; q.accin[a] = A[a]; q.acc[a] = nullptr; q.out[a] = Cb[a]; }
        LAUNCH(x, K_MOMP, launch_mom_pair<T>(1, q, x->Lo.LP, x->cur, x->rec));
    } else {
        for (int a = 0; a < 3; ++a) { m.us[a] = U[a]; m.acc[a] = A[a]; m.out[a] = B[a]; m.un[a] = nullptr; }
        LAUNCH(x, K_MOM, launch_mom_stage<T>(ST_FIRST, m, L, x->cur, x->rec));
        if (per_stage && (rc = project_stage(B, Cb))) return rc;
        for (int a = 0; a < 3; ++a) { m.us[a] = B[a]; m.un[a] = U[a]; m.out[a] = Cb[a]; }
        LAUNCH(x, K_MOM, launch_mom_stage<T>(ST_HALF, m, L, x->cur, x->rec));
        if (per_stage && (rc = project_stage(Cb, B))) return rc;
        for (int a = 0; a < 3; ++a) { m.us[a] = Cb[a]; m.out[a] = B[a]; }
        LAUNCH(x, K_MOM, launch_mom_stage<T>(ST_FULL, m, L, x->cur, x->rec));
        if (per_stage && (rc = project_stage(B, Cb))) return rc;
        for (int a = 0; a < 3; ++a) { m.us[a] = B[a]; m.un[a] = nullptr; m.out[a] = Cb[a]; }
        LAUNCH(x, K_MOM, launch_mom_stage<T>(ST_LAST, m, L, x->cur, x->rec));
    }
    // projection: u* in Cb -> projected velocity V
    const T* const us[3] = {Cb[0], Cb[1], Cb[2]};
    rc = project_div<T>(x, us);
    if (!rc && defer && !forked) rc = flush_scalar_half<T>(x);
    if (!rc) rc = project_solve<T>(x, us);
    if (!rc) rc = join_scalar_half(x);
    if (rc) return rc;
    const bool filt = x->P.filter != 0;
    T* V[3];
    projected_velocity<T>(x, V);
    rc = project_correct<T>(x, us, V, filt ? PartSoA{} : x->part);
    if (rc) return rc;
    if (filt) {
        FiltArgs<T> fa = {};
        for (int a = 0; a < 3; ++a) { fa.in[a] = V[a]; fa.out[a] = U[a]; }
        fa.nf = 3;
        fa.flags = x->flags;
        fa.g = x->g;
        fa.part = x->part;
        LAUNCH(x, K_FILT, launch_filter<T>(fa, x->Lo.LF, x->cur, x->rec));
    }
    AdvanceArgs av;
    av.part = x->part;
    av.np = filt ? x->Lo.LF.nblocks : x->Lo.LC.nblocks;
    av.sc = x->sc;
    LAUNCH(x, K_ADV, launch_advance(av, x->cur, x->rec));
    if (defer) {
        x->tail_pending = true;
    } else {
        rc = scalar_half<T>(x);
        if (rc) return rc;
    }
    if (!x->rec) x->host_step += 1;
    return DNSLAB_OK;
}

// Enqueue any deferred scalar work and order the main stream after it.
template <typename T>
int settle(dnslab_ctx* x) {
    int rc = flush_scalar_half<T>(x);
    if (!rc) rc = join_scalar_half(x);
    return rc;
}

void diag_copy(const DiagRec& r, dnslab_diag* d) {
    d->t = r.t;
    d->dt = r.dt;
    d->ke = r.ke;
    d->div_l2 = r.div_l2;
    d->co2_mass = r.co2_mass;
    d->co2_room_mean = r.co2_room_mean;
    d->cfl_max = r.cfl_max;
    d->step = r.step;
}

// Visit every cell with the bit set of its solid face neighbours
// (+x, -x, +y, -y, +z, -z) = (1, 2, 4, 8, 16, 32), periodic.
template <class F>
void for_each_cell_solid_neighbours(const uint8_t* beta, int nx, int ny, int nz, F&& visit) {
    for (int k = 0; k < nz; ++k) {
        const int kp = k + 1 == nz ? 0 : k + 1, km = k == 0 ? nz - 1 : k - 1;
        for (int j = 0; j < ny; ++j) {
            const int jp = j + 1 == ny ? 0 : j + 1, jm = j == 0 ? ny - 1 : j - 1;
            const size_t row = ((size_t)k * ny + j) * nx;
            const uint8_t* r0 = beta + row;
            const uint8_t* ryp = beta + ((size_t)k * ny + jp) * nx;
            const uint8_t* rym = beta + ((size_t)k * ny + jm) * nx;
            const uint8_t* rzp = beta + ((size_t)kp * ny + j) * nx;
            const uint8_t* rzm = beta + ((size_t)km * ny + j) * nx;
            for (int i = 0; i < nx; ++i) {
                const int ip = i + 1 == nx ? 0 : i + 1, im = i == 0 ? nx - 1 : i - 1;
                const unsigned m = (unsigned)(!r0[ip]) | (unsigned)(!r0[im]) << 1 | (unsigned)(!ryp[i]) << 2 |
                                   (unsigned)(!rym[i]) << 3 | (unsigned)(!rzp[i]) << 4 | (unsigned)(!rzm[i]) << 5;
                visit(row + i, m);
            }
        }
    }
}

int build_flags(dnslab_ctx* x, const uint8_t* beta_dev, const long long* fidx_host, int64_t nf,
                const uint8_t* room_dev) {
    const Grid& g = x->g;
    std::vector<uint8_t> beta((size_t)g.n), room;
    HIPCHK(x, hipMemcpy(beta.data(), beta_dev, (size_t)g.n, hipMemcpyDeviceToHost));
    if (room_dev) {
        room.resize((size_t)g.n);
        HIPCHK(x, hipMemcpy(room.data(), room_dev, (size_t)g.n, hipMemcpyDeviceToHost));
    }
    std::vector<uint8_t> fl((size_t)g.n, 0);
    std::vector<int> ibidx;
    std::vector<uint8_t> ibmask;
    bool any_solid = false;
    for (long long i = 0; i < g.n; ++i) {
        if (beta[i] > 1) return fail(x, DNSLAB_EINVAL, "beta must hold 0 or 1");
        if (!beta[i]) any_solid = true;
    }
    for_each_cell_solid_neighbours(beta.data(), g.nx, g.ny, g.nz, [&](size_t id, unsigned solid_nb) {
        uint8_t f = beta[id] ? F_FLUID : 0;
        if (room_dev ? room[id] != 0 : true) f |= F_ROOM;
        if (solid_nb) {
            f |= F_NEAR_SOLID;
            ibidx.push_back((int)id);
            ibmask.push_back((uint8_t)solid_nb);
        }
        fl[id] = f;
    });
    for (int64_t e = 0; e < nf; ++e) {
        const long long id = fidx_host[e];
        if (id < 0 || id >= g.n) return fail(x, DNSLAB_EINVAL, "forced index out of range");
        if (e > 0 && fidx_host[e - 1] >= id) return fail(x, DNSLAB_EINVAL, "forced indices must be sorted and unique");
        fl[id] |= F_FORCED;
    }
    HIPCHK(x, hipMemcpy(x->flags, fl.data(), (size_t)g.n, hipMemcpyHostToDevice));
    x->any_solid = any_solid;
    const size_t nib = ibidx.size();
    if (nib > 0) {
        const size_t b_idx = align_up(nib * sizeof(int), 256), b_mask = align_up(nib, 256);
        x->ib_buf = dev_alloc(x->da, b_idx + b_mask + nib * x->Lo.esz);
        if (!x->ib_buf) return fail(x, DNSLAB_ENOMEM, "allocation of the immersed-boundary list failed");
        char* b = (char*)x->ib_buf;
        HIPCHK(x, hipMemcpy(b, ibidx.data(), nib * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(x, hipMemcpy(b + b_idx, ibmask.data(), nib, hipMemcpyHostToDevice));
        x->ib.idx = (const int*)b;
        x->ib.mask = (const uint8_t*)(b + b_idx);
        x->ib_r0 = b + b_idx + b_mask;
    }
    x->ib.n = (int)nib;
    return DNSLAB_OK;
}

template <typename T>
int upload_tables(dnslab_ctx* x) {
    const Grid& g = x->g;
    const int m = x->Lo.m;
    std::vector<C2<T>> h;
    std::vector<long double> re, im;
    auto push = [&](int n, int count) {
        twiddles(n, re, im, count);
        for (int j = 0; j < count; ++j) h.push_back(C2<T>{(T)re[j], (T)im[j]});
    };
    push(m, m);
    push(g.ny, g.ny);
    push(g.nz, g.nz);
    push(g.nx, m + 1);
    HIPCHK(x, hipMemcpy(x->wx, h.data(), h.size() * sizeof(C2<T>), hipMemcpyHostToDevice));
    std::vector<double> s2((size_t)(m + 1 + g.ny + g.nz));
    sin2_table(g.nx, m + 1, g.d[0], s2.data());
    sin2_table(g.ny, g.ny, g.d[1], s2.data() + m + 1);
    sin2_table(g.nz, g.nz, g.d[2], s2.data() + m + 1 + g.ny);
    HIPCHK(x, hipMemcpy(x->sx2, s2.data(), s2.size() * sizeof(double), hipMemcpyHostToDevice));
    return DNSLAB_OK;
}

// Capture k whole steps (each step's deferred scalar half included and settled
// at the end) into an executable graph.  Nothing runs during capture; the host
// step counter is restored afterwards.
template <typename T>
int capture_steps(dnslab_ctx* x, int k) {
    if (x->gexec) {
        HIPCHK(x, hipGraphExecDestroy(x->gexec));
        x->gexec = nullptr;
    }
    const long long hs = x->host_step;
    HIPCHK(x, hipStreamBeginCapture(x->stream, hipStreamCaptureModeThreadLocal));
    int rc = DNSLAB_OK;
    for (int s = 0; s < k && !rc; ++s) rc = one_step<T>(x);
    if (!rc) rc = settle<T>(x);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(x->stream, &g);
    x->host_step = hs;
    x->tail_pending = false;
    x->join_pending = false;
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : fail(x, DNSLAB_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    const hipError_t e2 = hipGraphInstantiate(&x->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        x->gexec = nullptr;
        return fail(x, DNSLAB_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e2));
    }
    x->gexec_steps = k;
    return DNSLAB_OK;
}

template <typename T>
int run_steps(dnslab_ctx* x, int nsteps) {
    int rc = DNSLAB_OK;
    const int k = x->graph_steps;
    if (k > 0 && nsteps >= k && !x->rec && x->prof_kid == K_NONE) {
        // first-step work (Courant rate, second stream) happens outside the graph
        rc = ensure_rate<T>(x);
        if (!rc && x->overlap) rc = ensure_aux(x);
        if (!rc && (!x->gexec || x->gexec_steps != k)) rc = capture_steps<T>(x, k);
        while (!rc && nsteps >= k) {
            const hipError_t e = hipGraphLaunch(x->gexec, x->stream);
            if (e != hipSuccess) return fail(x, DNSLAB_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
            x->host_step += k;
            nsteps -= k;
        }
    }
    for (int s = 0; s < nsteps && !rc; ++s) rc = one_step<T>(x);
    const int rc2 = settle<T>(x);
    return rc ? rc : rc2;
}

int check_ctx(dnslab_ctx* x) {
    if (!x) return fail(nullptr, DNSLAB_EINVAL, "ctx is NULL");
    return DNSLAB_OK;
}

}  // namespace

namespace {
template <typename T>
int mom_rhs(dnslab_ctx* x, const void* u, const void* v, const void* w, void* fu, void* fv, void* fw) {
    MomArgs<T> m = {};
    m.us[0] = (const T*)u; m.us[1] = (const T*)v; m.us[2] = (const T*)w;
    m.out[0] = (T*)fu; m.out[1] = (T*)fv; m.out[2] = (T*)fw;
    m.flags = x->flags;
    m.frc = forcing_of<T>(x);
    m.nu = x->P.nu;
    for (int a = 0; a < 3; ++a) m.body[a] = x->P.body[a];
    m.g = x->g;
    LAUNCH(x, K_MOM, launch_mom_stage<T>(ST_RHS, m, x->Lo.L, x->cur, x->rec));
    return DNSLAB_OK;
}
template <typename T>
int sca_rhs(dnslab_ctx* x, const void* c, const void* u, const void* v, const void* w, void* out) {
    ScaArgs<T> s = {};
    s.cs = (const T*)c;
    s.u[0] = (const T*)u; s.u[1] = (const T*)v; s.u[2] = (const T*)w;
    s.out = (T*)out;
    s.flags = x->flags;
    s.frc = forcing_of<T>(x);
    s.alpha = x->P.alpha_c;
    s.g = x->g;
    LAUNCH(x, K_SCA, launch_sca_stage<T>(ST_RHS, s, x->Lo.L, x->cur, x->rec));
    return DNSLAB_OK;
}
template <typename T>
int filt1(dnslab_ctx* x, const void* f, void* out) {
    FiltArgs<T> a = {};
    a.in[0] = (const T*)f;
    a.out[0] = (T*)out;
    a.nf = 1;
    a.flags = x->flags;
    a.g = x->g;
    LAUNCH(x, K_FILT, launch_filter<T>(a, x->Lo.LF, x->cur, x->rec));
    return DNSLAB_OK;
}
}  // namespace

// ---------------------------------------------------------------------------
// The allocation-free Poisson solve keeps its spectrum and tables in one
// file-scope device array.  In host code `scratch` only stands in for the
// symbol: its device address (one copy per GPU) is looked up once per device
// with hipGetSymbolAddress, and that address is what the kernels receive.
static __device__ __align__(256) unsigned char scratch[DNSLAB_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`.
int noalloc_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, DNSLAB_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(nullptr, DNSLAB_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, DNSLAB_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return DNSLAB_OK;
}

// Scratch layout of the allocation-free solve: the spectrum as a context
// stores it, then the twiddle tables, then the symbol tables.
struct NoallocLayout {
    size_t off_w, off_s2, total;
};

NoallocLayout noalloc_layout(const Layout& Lo, const dnslab_params* P) {
    const size_t csz = 2 * Lo.esz;
    NoallocLayout N;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
    take((size_t)Lo.sx * P->ny * P->nz * csz);
    N.off_w = take((size_t)(2 * Lo.m + 1 + P->ny + P->nz) * csz);
    N.off_s2 = take((size_t)(Lo.m + 1 + P->ny + P->nz) * sizeof(double));
    N.total = off;
    return N;
}

template <typename T>
int poisson_noalloc(const dnslab_params* P, const T* r, T* pout) {
    const Layout Lo = make_layout(P, 0);
    const Grid g = make_grid(P);
    const NoallocLayout N = noalloc_layout(Lo, P);
    if (N.total > (size_t)DNSLAB_NOALLOC_SCRATCH_BYTES)
        return fail(nullptr, DNSLAB_EINVAL,
                    "grid " + std::to_string(P->nx) + "x" + std::to_string(P->ny) + "x" + std::to_string(P->nz) +
                        " needs " + std::to_string(N.total) + " bytes of scratch; the allocation-free solve holds " +
                        std::to_string((size_t)DNSLAB_NOALLOC_SCRATCH_BYTES));
    void* base = nullptr;
    if (int rc = noalloc_scratch(&base)) return rc;
    char* b = (char*)base;
    const FFTArgs<T> a = fft_args_of<T>(Lo, g, b, b + N.off_w, (const double*)(b + N.off_s2));
    const hipStream_t s = (hipStream_t)P->stream;
    hipError_t e = launch_fft_tables<T>((C2<T>*)(b + N.off_w), (double*)(b + N.off_s2), g, s);
    if (e == hipSuccess) e = launch_fft_x_fwd<T>(a, r, s);
    if (e == hipSuccess) {
        if (Lo.yz) {
            e = launch_fft_yz_solve<T>(a, s);
        } else {
            if (g.ny > 1) e = launch_fft_y<T>(a, false, s);
            if (e == hipSuccess) e = launch_fft_z_solve<T>(a, s);
            if (e == hipSuccess && g.ny > 1) e = launch_fft_y<T>(a, true, s);
        }
    }
    if (e == hipSuccess) e = launch_fft_x_inv<T>(a, pout, s);
    if (e != hipSuccess) return fail(nullptr, DNSLAB_EHIP, std::string("launch: ") + hipGetErrorString(e));
    return DNSLAB_OK;
}

}  // namespace

extern "C" {

int dnslab_workspace_bytes(const dnslab_params* params, size_t* out_bytes) {
    try {
        std::string why;
        int rc = validate(params, why);
        if (rc) return fail(nullptr, rc, why);
        if (!out_bytes) return fail(nullptr, DNSLAB_EINVAL, "out_bytes is NULL");
        *out_bytes = make_layout(params, 0).total;
        return DNSLAB_OK;
    } catch (...) {
        return fail(nullptr, DNSLAB_ENOMEM, "host allocation failed");
    }
}

int dnslab_init(const dnslab_params* params, const uint8_t* beta_dev, int64_t n_forced,
                const int64_t* forced_idx_dev, const double* forced_S_dev, const double* forced_uset_dev,
                const double* forced_cset_dev, const uint8_t* room_mask_dev, void* u, void* v, void* w, void* p,
                void* c, dnslab_ctx** out) {
    dnslab_ctx* x = nullptr;
    try {
        std::string why;
        int rc = validate(params, why);
        if (rc) return fail(nullptr, rc, why);
        if (!out || !beta_dev || !u || !v || !w || !p || !c) return fail(nullptr, DNSLAB_EINVAL, "NULL pointer argument");
        if (n_forced < 0 || n_forced > (1 << 30)) return fail(nullptr, DNSLAB_EINVAL, "bad n_forced");
        if (n_forced > 0 && (!forced_idx_dev || !forced_S_dev || !forced_uset_dev || !forced_cset_dev))
            return fail(nullptr, DNSLAB_EINVAL, "NULL forcing array");
        *out = nullptr;
        x = new dnslab_ctx();
        x->P = *params;
        x->da = alloc_of(params);
        x->stream = (hipStream_t)params->stream;
        x->cur = x->stream;
        x->overlap = DNSLAB_OVERLAP != 0;
        x->g = make_grid(params);
        x->Lo = make_layout(params, (int)n_forced);
        x->u = u; x->v = v; x->w = w; x->p = p; x->c = c;
        x->prof_kid = K_NONE;
        x->nforced = (int)n_forced;
        x->ws = dev_alloc(x->da, x->Lo.total);
        if (!x->ws) {
            delete x;
            return fail(nullptr, DNSLAB_ENOMEM, "allocation of the workspace failed");
        }
        char* base = (char*)x->ws;
        const Layout& Lo = x->Lo;
        x->flags = (uint8_t*)(base + Lo.off_flags);
        for (int i = 0; i < Lo.nfields; ++i) x->f[i] = base + Lo.off_fields + (size_t)i * Lo.n * Lo.esz;
        x->spec = base + Lo.off_spec;
        const size_t csz = 2 * Lo.esz;
        x->wx = base + Lo.off_tw;
        x->wy = (char*)x->wx + (size_t)Lo.m * csz;
        x->wz = (char*)x->wy + (size_t)params->ny * csz;
        x->tw = (char*)x->wz + (size_t)params->nz * csz;
        x->sx2 = (double*)(base + Lo.off_s2);
        x->sy2 = x->sx2 + Lo.m + 1;
        x->sz2 = x->sy2 + params->ny;
        x->fidx = (long long*)(base + Lo.off_forced);
        x->fS = (double*)(x->fidx + Lo.nforced_cap);
        x->fuset = x->fS + Lo.nforced_cap;
        x->fcset = x->fuset + 3 * (size_t)Lo.nforced_cap;
        x->part = PartSoA{(double*)(base + Lo.off_part), Lo.nparts};
        x->sc = (StepScalars*)(base + Lo.off_sc);
        x->ring = (DiagRec*)(base + Lo.off_ring);
        if (hipHostMalloc((void**)&x->pinned, RING_CAP * sizeof(DiagRec), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&x->pinned_sc, sizeof(StepScalars), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            dnslab_destroy(x);
            return fail(nullptr, DNSLAB_ENOMEM, "hipHostMalloc failed");
        }
        std::vector<long long> fidx_h((size_t)n_forced);
        if (n_forced > 0) {
            if (hipMemcpy(fidx_h.data(), forced_idx_dev, n_forced * sizeof(long long), hipMemcpyDeviceToHost) != hipSuccess) {
                dnslab_destroy(x);
                return fail(nullptr, DNSLAB_EHIP, "reading forced indices failed");
            }
        }
        rc = build_flags(x, beta_dev, fidx_h.data(), n_forced, room_mask_dev);
        if (rc == DNSLAB_OK && n_forced > 0) {
            const hipStream_t st = x->stream;
            if (hipMemcpyAsync(x->fidx, forced_idx_dev, n_forced * sizeof(long long), hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(x->fS, forced_S_dev, n_forced * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(x->fuset, forced_uset_dev, 3 * n_forced * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(x->fcset, forced_cset_dev, n_forced * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
                rc = fail(x, DNSLAB_EHIP, "copying forcing arrays failed");
        }
        if (rc == DNSLAB_OK) rc = Lo.esz == 8 ? upload_tables<double>(x) : upload_tables<float>(x);
        if (rc == DNSLAB_OK) {
            StepScalars s = {};
            s.dt_fixed = params->dt_fixed > 0 ? params->dt_fixed : 0.0;
            s.cfl = params->cfl;
            const double dmin = std::min(x->g.d[0], std::min(x->g.d[1], x->g.d[2]));
            s.rate_floor = params->dt_fixed > 0 ? 0.0 : params->u_ref / dmin;
            s.dt = s.dt_fixed;
            if (hipMemcpy(x->sc, &s, sizeof(s), hipMemcpyHostToDevice) != hipSuccess)
                rc = fail(x, DNSLAB_EHIP, "uploading step scalars failed");
        }
        if (rc == DNSLAB_OK) rc = Lo.esz == 8 ? ensure_rate<double>(x) : ensure_rate<float>(x);
        if (rc == DNSLAB_OK && hipStreamSynchronize(x->stream) != hipSuccess) rc = fail(x, DNSLAB_EHIP, "sync failed");
        if (rc != DNSLAB_OK) {
            g_thread_err = x->err.empty() ? g_thread_err : x->err;
            dnslab_destroy(x);
            return rc;
        }
        *out = x;
        return DNSLAB_OK;
    } catch (...) {
        if (x) dnslab_destroy(x);
        return fail(nullptr, DNSLAB_ENOMEM, "host allocation failed");
    }
}

int dnslab_step(dnslab_ctx* x, int32_t nsteps, dnslab_diag* diag) {
    if (int rc = check_ctx(x)) return rc;
    try {
        if (nsteps < 0) return fail(x, DNSLAB_EINVAL, "nsteps < 0");
        int rc = x->Lo.esz == 8 ? run_steps<double>(x, nsteps) : run_steps<float>(x, nsteps);
        if (rc) return rc;
        if (diag) {
            if (x->host_step == 0) return fail(x, DNSLAB_ESTATE, "no step taken yet");
            const long long slot = (x->host_step - 1) % RING_CAP;
            HIPCHK(x, hipMemcpyAsync(x->pinned, x->ring + slot, sizeof(DiagRec), hipMemcpyDeviceToHost, x->stream));
            HIPCHK(x, hipMemcpyAsync(x->pinned_sc, x->sc, sizeof(StepScalars), hipMemcpyDeviceToHost, x->stream));
            HIPCHK(x, hipStreamSynchronize(x->stream));
            diag_copy(x->pinned[0], diag);
            if (x->pinned_sc->nonfinite || x->pinned_sc->nonfinite_diag)
                return fail(x, DNSLAB_ENONFINITE, "non-finite diagnostics");
        }
        return DNSLAB_OK;
    } catch (...) {
        return fail(x, DNSLAB_ENOMEM, "host allocation failed");
    }
}

int dnslab_read_diags(dnslab_ctx* x, int32_t n, dnslab_diag* out) {
    if (int rc = check_ctx(x)) return rc;
    if (n < 0 || n > RING_CAP || (n > 0 && !out)) return fail(x, DNSLAB_EINVAL, "bad n or out");
    if (n > x->host_step) return fail(x, DNSLAB_ESTATE, "fewer steps taken than requested");
    HIPCHK(x, hipMemcpyAsync(x->pinned, x->ring, RING_CAP * sizeof(DiagRec), hipMemcpyDeviceToHost, x->stream));
    HIPCHK(x, hipStreamSynchronize(x->stream));
    for (int i = 0; i < n; ++i) {
        const long long st = x->host_step - n + i;   // 0-based step index
        diag_copy(x->pinned[st % RING_CAP], out + i);
    }
    return DNSLAB_OK;
}

int dnslab_poisson(dnslab_ctx* x, const void* rhs, void* p) {
    if (int rc = check_ctx(x)) return rc;
    if (!rhs || !p) return fail(x, DNSLAB_EINVAL, "NULL pointer");
    if (x->Lo.esz == 8) return poisson_solve<double>(x, (const double*)rhs, (double*)p);
    return poisson_solve<float>(x, (const float*)rhs, (float*)p);
}

int dnslab_poisson_noalloc(const dnslab_params* params, const void* rhs, void* p) {
    try {
        std::string why;
        int rc = validate(params, why);
        if (rc) return fail(nullptr, rc, why);
        if (!rhs || !p) return fail(nullptr, DNSLAB_EINVAL, "NULL pointer");
        if (params->precision == DNSLAB_FP64) return poisson_noalloc<double>(params, (const double*)rhs, (double*)p);
        return poisson_noalloc<float>(params, (const float*)rhs, (float*)p);
    } catch (...) {
        return fail(nullptr, DNSLAB_ENOMEM, "host allocation failed");
    }
}

int dnslab_project(dnslab_ctx* x, void* u, void* v, void* w) {
    if (int rc = check_ctx(x)) return rc;
    if (!u || !v || !w) return fail(x, DNSLAB_EINVAL, "NULL pointer");
    x->rate_valid = false;
    if (x->Lo.esz == 8) {
        double* U[3] = {(double*)u, (double*)v, (double*)w};
        return project<double>(x, U, U);
    }
    float* U[3] = {(float*)u, (float*)v, (float*)w};
    return project<float>(x, U, U);
}

int dnslab_scalar_step(dnslab_ctx* x, double dt) {
    if (int rc = check_ctx(x)) return rc;
    if (!std::isfinite(dt)) return fail(x, DNSLAB_EINVAL, "dt not finite");
    if (x->Lo.esz == 8) {
        const double* U[3] = {(double*)x->u, (double*)x->v, (double*)x->w};
        return scalar_rk4<double>(x, U, nullptr, dt, (double*)x->c, PartSoA{}, PartSoA{});
    }
    const float* U[3] = {(float*)x->u, (float*)x->v, (float*)x->w};
    return scalar_rk4<float>(x, U, nullptr, dt, (float*)x->c, PartSoA{}, PartSoA{});
}


int dnslab_momentum_rhs(dnslab_ctx* x, const void* u, const void* v, const void* w, void* fu, void* fv, void* fw) {
    if (int rc = check_ctx(x)) return rc;
    if (!u || !v || !w || !fu || !fv || !fw) return fail(x, DNSLAB_EINVAL, "NULL pointer");
    return x->Lo.esz == 8 ? mom_rhs<double>(x, u, v, w, fu, fv, fw) : mom_rhs<float>(x, u, v, w, fu, fv, fw);
}

int dnslab_scalar_rhs(dnslab_ctx* x, const void* c, const void* u, const void* v, const void* w, void* out) {
    if (int rc = check_ctx(x)) return rc;
    if (!c || !u || !v || !w || !out) return fail(x, DNSLAB_EINVAL, "NULL pointer");
    return x->Lo.esz == 8 ? sca_rhs<double>(x, c, u, v, w, out) : sca_rhs<float>(x, c, u, v, w, out);
}

int dnslab_filter(dnslab_ctx* x, const void* f, void* out) {
    if (int rc = check_ctx(x)) return rc;
    if (!f || !out || f == out) return fail(x, DNSLAB_EINVAL, "NULL or aliased pointer");
    return x->Lo.esz == 8 ? filt1<double>(x, f, out) : filt1<float>(x, f, out);
}

int dnslab_set_time(dnslab_ctx* x, double t, int64_t step) {
    if (int rc = check_ctx(x)) return rc;
    if (!std::isfinite(t) || step < 0) return fail(x, DNSLAB_EINVAL, "bad t or step");
    HIPCHK(x, hipMemcpyAsync(x->pinned_sc, x->sc, sizeof(StepScalars), hipMemcpyDeviceToHost, x->stream));
    HIPCHK(x, hipStreamSynchronize(x->stream));
    StepScalars s = *x->pinned_sc;
    s.t = t;
    s.step = step;
    s.nonfinite = 0;
    s.nonfinite_diag = 0;
    *x->pinned_sc = s;
    HIPCHK(x, hipMemcpyAsync(x->sc, x->pinned_sc, sizeof(StepScalars), hipMemcpyHostToDevice, x->stream));
    x->host_step = step;
    x->rate_valid = false;
    int rc = x->Lo.esz == 8 ? ensure_rate<double>(x) : ensure_rate<float>(x);
    if (rc) return rc;
    HIPCHK(x, hipStreamSynchronize(x->stream));
    return DNSLAB_OK;
}

void dnslab_destroy(dnslab_ctx* x) {
    if (!x) return;
    (void)hipStreamSynchronize(x->stream);
    if (x->aux) {
        (void)hipStreamSynchronize(x->aux);
        (void)hipStreamDestroy(x->aux);
        (void)hipEventDestroy(x->ev_fork);
        (void)hipEventDestroy(x->ev_join);
    }
    if (x->gexec) (void)hipGraphExecDestroy(x->gexec);
    for (hipEvent_t e : x->ev) (void)hipEventDestroy(e);
    dev_free(x->da, x->ws);
    dev_free(x->da, x->ib_buf);
    dev_free(x->da, x->hist_dev);
    if (x->hist_host) (void)hipHostFree(x->hist_host);
    dev_free(x->da, x->psort_buf);
    if (x->pinned) (void)hipHostFree(x->pinned);
    if (x->pinned_sc) (void)hipHostFree(x->pinned_sc);
    delete x;
}

const char* dnslab_last_error(const dnslab_ctx* x) {
    if (x) return x->err.c_str();
    return g_thread_err.c_str();
}

int dnslab_profile_enable(dnslab_ctx* x, const char* name) {
    if (int rc = check_ctx(x)) return rc;
    int kid = K_NONE;
    if (name)
        for (int k = 0; k < K_COUNT; ++k)
            if (std::strcmp(name, kKernelNames[k]) == 0) kid = k;
    if (name && kid == K_NONE) return fail(x, DNSLAB_EINVAL, "unknown kernel name");
    int rc = prof_flush(x);
    if (rc) return rc;
    if (x->ev.empty() && kid != K_NONE) {
        try {
            x->ev.resize(PROF_POOL);
        } catch (...) {
            return fail(x, DNSLAB_ENOMEM, "host allocation failed");
        }
        for (auto& e : x->ev) HIPCHK(x, hipEventCreate(&e));
    }
    x->prof_kid = kid;
    x->prof_ms = 0;
    x->prof_n = 0;
    return DNSLAB_OK;
}

int dnslab_particles_step(dnslab_ctx* x, int64_t n, double* pos, double* vel, const double* diam,
                          const dnslab_particle_params* pp, double dt) {
    if (int rc = check_ctx(x)) return rc;
    if (n < 0 || n >= (1LL << 40)) return fail(x, DNSLAB_EINVAL, "bad particle count");
    if (!pp || (n > 0 && (!pos || !vel || !diam))) return fail(x, DNSLAB_EINVAL, "NULL pointer");
    if (!(pp->rho_p > 0) || !(pp->rho_f > 0) || !std::isfinite(pp->g[0]) || !std::isfinite(pp->g[1]) ||
        !std::isfinite(pp->g[2]) || !std::isfinite(dt))
        return fail(x, DNSLAB_EINVAL, "bad particle parameters");
    if (!(x->P.nu > 0)) return fail(x, DNSLAB_EINVAL, "particles need nu > 0");
    auto fill = [&](auto& a) {
        a.g = x->g;
        a.box[0] = x->P.lx; a.box[1] = x->P.ly; a.box[2] = x->P.lz;
        a.px = pos; a.py = pos + n; a.pz = pos + 2 * n;
        a.vx = vel; a.vy = vel + n; a.vz = vel + 2 * n;
        a.diam = diam;
        a.n = n;
        a.nu = x->P.nu;
        a.rho_p = pp->rho_p;
        a.rho_f = pp->rho_f;
        for (int i = 0; i < 3; ++i) a.g_acc[i] = pp->g[i];
        a.dtp = dt > 0 ? nullptr : &x->sc->last_dt;
        a.dt = dt;
    };
    if (x->Lo.esz == 8) {
        ParticleArgs<double> a;
        a.u = (const double*)x->u; a.v = (const double*)x->v; a.w = (const double*)x->w;
        fill(a);
        LAUNCH(x, K_PART, launch_particles<double>(a, x->stream));
    } else {
        ParticleArgs<float> a;
        a.u = (const float*)x->u; a.v = (const float*)x->v; a.w = (const float*)x->w;
        fill(a);
        LAUNCH(x, K_PART, launch_particles<float>(a, x->stream));
    }
    return DNSLAB_OK;
}

int dnslab_particles_sort(dnslab_ctx* x, int64_t n, double* pos, double* vel, double* diam) {
    if (int rc = check_ctx(x)) return rc;
    if (n < 0 || n > particle_sort_max()) return fail(x, DNSLAB_EINVAL, "bad particle count (0 <= n <= 2^28)");
    if (n > 0 && (!pos || !vel || !diam)) return fail(x, DNSLAB_EINVAL, "NULL pointer");
    if (n == 0) return DNSLAB_OK;
    size_t sort_bytes = 0;
    HIPCHK(x, particle_sort_bytes(n, &sort_bytes));
    const size_t b_key = align_up((size_t)n * sizeof(unsigned), 256), b_tmp = align_up((size_t)n * sizeof(double), 256);
    const size_t need = 4 * b_key + b_tmp + align_up(sort_bytes, 256);
    if (need > x->psort_bytes) {
        if (x->psort_buf) {
            // an earlier sort on the stream may still use the old scratch
            HIPCHK(x, hipStreamSynchronize(x->stream));
            dev_free(x->da, x->psort_buf);
            x->psort_buf = nullptr;
            x->psort_bytes = 0;
        }
        x->psort_buf = dev_alloc(x->da, need);
        if (!x->psort_buf) return fail(x, DNSLAB_ENOMEM, "particle sort scratch");
        x->psort_bytes = need;
    }
    char* b = (char*)x->psort_buf;
    ParticleSortScratch sc;
    sc.keys[0] = (unsigned*)b;
    sc.keys[1] = (unsigned*)(b + b_key);
    sc.vals[0] = (unsigned*)(b + 2 * b_key);
    sc.vals[1] = (unsigned*)(b + 3 * b_key);
    sc.tmp = (double*)(b + 4 * b_key);
    sc.sort_tmp = b + 4 * b_key + b_tmp;
    sc.sort_bytes = sort_bytes;
    HIPCHK(x, sort_particles(x->g, n, pos, vel, diam, sc, x->stream));
    return DNSLAB_OK;
}

int dnslab_co2_histogram(dnslab_ctx* x, int32_t nbins, double lo, double hi, int64_t* counts_host) {
    if (int rc = check_ctx(x)) return rc;
    if (nbins < 1 || nbins > HIST_MAX_BINS || !(lo < hi) || !std::isfinite(lo) || !std::isfinite(hi) || !counts_host)
        return fail(x, DNSLAB_EINVAL, "bad histogram arguments");
    if (!x->hist_dev) {
        x->hist_dev = (unsigned long long*)dev_alloc(x->da, HIST_MAX_BINS * sizeof(unsigned long long));
        if (!x->hist_dev) return fail(x, DNSLAB_ENOMEM, "histogram counters");
    }
    if (!x->hist_host) {
        if (hipHostMalloc((void**)&x->hist_host, HIST_MAX_BINS * sizeof(unsigned long long), hipHostMallocDefault) !=
            hipSuccess) {
            (void)hipGetLastError();
            x->hist_host = nullptr;
            return fail(x, DNSLAB_ENOMEM, "histogram host buffer");
        }
    }
    hipError_t e;
    if (x->Lo.esz == 8) {
        HistArgs<double> a = {(const double*)x->c, x->flags, x->g.n, nbins, lo, hi, x->hist_dev};
        e = launch_histogram<double>(a, x->stream);
    } else {
        HistArgs<float> a = {(const float*)x->c, x->flags, x->g.n, nbins, lo, hi, x->hist_dev};
        e = launch_histogram<float>(a, x->stream);
    }
    if (e != hipSuccess) return fail(x, DNSLAB_EHIP, std::string("histogram: ") + hipGetErrorString(e));
    HIPCHK(x, hipMemcpyAsync(x->hist_host, x->hist_dev, nbins * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             x->stream));
    HIPCHK(x, hipStreamSynchronize(x->stream));
    for (int b = 0; b < nbins; ++b) counts_host[b] = (int64_t)x->hist_host[b];
    return DNSLAB_OK;
}

int dnslab_accumulate(dnslab_ctx* x, double* sums_dev) {
    if (int rc = check_ctx(x)) return rc;
    if (!sums_dev) return fail(x, DNSLAB_EINVAL, "NULL pointer");
    hipError_t e;
    if (x->Lo.esz == 8) {
        AccArgs<double> a = {{(const double*)x->u, (const double*)x->v, (const double*)x->w, (const double*)x->p,
                              (const double*)x->c}, sums_dev, x->g.n};
        e = launch_accumulate<double>(a, x->stream);
    } else {
        AccArgs<float> a = {{(const float*)x->u, (const float*)x->v, (const float*)x->w, (const float*)x->p,
                             (const float*)x->c}, sums_dev, x->g.n};
        e = launch_accumulate<float>(a, x->stream);
    }
    if (e != hipSuccess) return fail(x, DNSLAB_EHIP, std::string("accumulate: ") + hipGetErrorString(e));
    return DNSLAB_OK;
}

int dnslab_body_force(dnslab_ctx* x, const int32_t box[6], double* out_dev) {
    if (int rc = check_ctx(x)) return rc;
    if (!box || !out_dev) return fail(x, DNSLAB_EINVAL, "NULL pointer");
    const int nn[3] = {x->g.nx, x->g.ny, x->g.nz};
    for (int a = 0; a < 3; ++a)
        if (box[2 * a] < 0 || box[2 * a] >= box[2 * a + 1] || box[2 * a + 1] > nn[a])
            return fail(x, DNSLAB_EINVAL, "box outside the grid or empty");
    hipError_t e;
    auto fill = [&](auto& a) {
        for (int q = 0; q < 6; ++q) a.box[q] = box[q];
        a.flags = x->flags;
        a.g = x->g;
        a.nu = x->P.nu;
        a.sc = x->sc;
        a.out = out_dev;
    };
    if (x->Lo.esz == 8) {
        ForceArgs<double> a;
        a.vel[0] = (const double*)x->u; a.vel[1] = (const double*)x->v; a.vel[2] = (const double*)x->w;
        a.p = (const double*)x->p;
        fill(a);
        e = launch_body_force<double>(a, x->stream);
    } else {
        ForceArgs<float> a;
        a.vel[0] = (const float*)x->u; a.vel[1] = (const float*)x->v; a.vel[2] = (const float*)x->w;
        a.p = (const float*)x->p;
        fill(a);
        e = launch_body_force<float>(a, x->stream);
    }
    if (e != hipSuccess) return fail(x, DNSLAB_EHIP, std::string("body force: ") + hipGetErrorString(e));
    return DNSLAB_OK;
}

int dnslab_set_graph_steps(dnslab_ctx* x, int32_t k) {
    if (int rc = check_ctx(x)) return rc;
    if (k < 0 || k > 4096) return fail(x, DNSLAB_EINVAL, "graph steps out of range");
    if (k > 0 && !x->stream) return fail(x, DNSLAB_EINVAL, "graph replay needs a non-NULL stream");
    x->graph_steps = k;
    return DNSLAB_OK;
}

int dnslab_set_overlap(dnslab_ctx* x, int32_t enable) {
    if (int rc = check_ctx(x)) return rc;
    if (enable != 0 && enable != 1) return fail(x, DNSLAB_EINVAL, "enable must be 0 or 1");
    try {
        // the deferred scalar half of the last step is enqueued and joined first
        int rc = x->Lo.esz == 8 ? settle<double>(x) : settle<float>(x);
        if (rc) return rc;
    } catch (...) {
        return fail(x, DNSLAB_ENOMEM, "host allocation failed");
    }
    if (x->overlap != (enable != 0) && x->gexec) {
        HIPCHK(x, hipGraphExecDestroy(x->gexec));   // captured with the other schedule
        x->gexec = nullptr;
    }
    x->overlap = enable != 0;
    return DNSLAB_OK;
}

int dnslab_set_stage_pairs(dnslab_ctx* x, int32_t mode) {
    if (int rc = check_ctx(x)) return rc;
    if (mode < -1 || mode > 1) return fail(x, DNSLAB_EINVAL, "mode must be -1, 0 or 1");
    try {
        int rc = x->Lo.esz == 8 ? settle<double>(x) : settle<float>(x);
        if (rc) return rc;
    } catch (...) {
        return fail(x, DNSLAB_ENOMEM, "host allocation failed");
    }
    if (x->pairs_mode != mode && x->gexec) {
        HIPCHK(x, hipGraphExecDestroy(x->gexec));   // captured with the other kernels
        x->gexec = nullptr;
    }
    x->pairs_mode = mode;
    return DNSLAB_OK;
}

int dnslab_set_fft_pipeline(dnslab_ctx* x, int32_t mode) {
    if (int rc = check_ctx(x)) return rc;
    if (mode < -1 || mode > 1) return fail(x, DNSLAB_EINVAL, "mode must be -1, 0 or 1");
    try {
        int rc = x->Lo.esz == 8 ? settle<double>(x) : settle<float>(x);
        if (rc) return rc;
    } catch (...) {
        return fail(x, DNSLAB_ENOMEM, "host allocation failed");
    }
    if (x->fft_pipe_mode != mode && x->gexec) {
        HIPCHK(x, hipGraphExecDestroy(x->gexec));   // captured with the other kernels
        x->gexec = nullptr;
    }
    x->fft_pipe_mode = mode;
    return DNSLAB_OK;
}

int dnslab_profile_read(dnslab_ctx* x, double* total_ms, int64_t* launches) {
    if (int rc = check_ctx(x)) return rc;
    int rc = prof_flush(x);
    if (rc) return rc;
    if (total_ms) *total_ms = x->prof_ms;
    if (launches) *launches = x->prof_n;
    return DNSLAB_OK;
}

}  // extern "C"

// ===========================================================================
// Serving pool: many resident scenarios advanced together.  Each scenario is
// an ordinary context with its own state and workspace.  The pool records the
// launch sequence of one step of every active scenario once (nothing is
// issued while recording), groups scenarios whose sequences match, and
// replays each position of a group's sequence as one batched launch over all
// its scenarios.  A scenario's blocks compute exactly what its own launches
// would, so its result is the same alone and in any mix.
// ===========================================================================
namespace {

struct PoolSlot {
    dnslab_ctx* ctx = nullptr;
    void* state = nullptr;
    size_t bytes = 0;
    long long target = 0, done = 0;
    bool used = false;
};

struct BatchPos {
    int kind;
    dim3 block;
    size_t lds;
    unsigned total;
    int ns;
    size_t tab_off, st_off;
};

struct BatchGroup {
    std::vector<int> slots;
    std::vector<BatchPos> seq;
    // Direct groups issue each scenario's own plain step: a group of one (no
    // batched-table lookups), or scenarios large enough to fill the GPU alone,
    // which then also overlap their scalar half with their next pressure solve.
    bool direct = false;
};
constexpr long long POOL_DIRECT_CELLS = 1LL << 20;
// Budget reserved per scenario for its share of the batched launch tables
// (about 70 launch records of at most ~0.5 KB per step sequence).
constexpr size_t POOL_TABLE_RESERVE = 64 * 1024;

}  // namespace

struct dnslab_pool {
    size_t budget = 0, used = 0;          // used: scenarios (with their table reserve) + the staging buffer
    DevAlloc da;                          // device memory of every scenario and of the pool itself
    int precision = 0;
    hipStream_t stream = nullptr;
    hipStream_t admit_stream = nullptr;   // init work of new scenarios, off the stepping stream
    void* stage = nullptr;                // device staging for admission inputs (kept: hipFree synchronises)
    size_t stage_cap = 0;
    std::vector<PoolSlot> slots;
    std::vector<BatchGroup> groups;
    std::vector<int> active_ids;
    bool dirty = true;
    void* tab_dev = nullptr;
    size_t tab_cap = 0;
    bool use_graph = false;
    hipGraphExec_t gexec = nullptr;       // one pool step, for the current groups
    // Groups (scenarios of one launch sequence) are independent of each other:
    // each step they run on separate streams, forked from and joined back into
    // the pool's stream, so that groups of different grid sizes fill each
    // other's idle time.
    std::vector<hipStream_t> gs;
    std::vector<hipEvent_t> gev;          // join events, one per group stream
    hipEvent_t fork_ev = nullptr;
    std::string err;
};

namespace {

int pfail(dnslab_pool* p, int code, const std::string& msg) {
    if (p) p->err = msg;
    else g_thread_err = msg;
    return code;
}

#define PHIP(pool, call)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return pfail(pool, DNSLAB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool is_stencil_kind(int kind) { return (kind >> 8) < KK_IB; }

// Record one step of every active slot and build the batched tables.
int pool_rebuild(dnslab_pool* P, const std::vector<int>& active) {
    PHIP(P, hipStreamSynchronize(P->stream));   // old tables may still be in use
    std::vector<std::vector<LaunchRecord>> recs(active.size());
    for (size_t q = 0; q < active.size(); ++q) {
        dnslab_ctx* x = P->slots[active[q]].ctx;
        Recorder r;
        x->rec = &r;
        const int rc = x->Lo.esz == 8 ? one_step<double>(x) : one_step<float>(x);
        x->rec = nullptr;
        if (rc) return pfail(P, rc, "recording a step failed: " + x->err);
        recs[q] = std::move(r.recs);
    }
    // group slots by sequence signature
    auto sig = [&](size_t q) {
        std::vector<long long> v;
        for (const LaunchRecord& l : recs[q]) {
            long long key = (long long)l.kind << 32;
            if (is_stencil_kind(l.kind)) key |= (long long)(l.block.x << 16 | l.block.y);
            v.push_back(key);
            v.push_back((long long)l.rec.size());
        }
        return v;
    };
    std::vector<std::vector<long long>> sigs;
    P->groups.clear();
    for (size_t q = 0; q < active.size(); ++q) {
        const std::vector<long long> s = sig(q);
        size_t g = 0;
        for (; g < sigs.size(); ++g)
            if (sigs[g] == s) break;
        if (g == sigs.size()) {
            sigs.push_back(s);
            P->groups.emplace_back();
        }
        P->groups[g].slots.push_back((int)q);   // index into active/recs for now
    }
    // lay out the tables
    std::vector<unsigned char> host;
    auto put = [&](const void* src, size_t n) {
        const size_t off = align_up(host.size(), 256);
        host.resize(off + n);
        std::memcpy(host.data() + off, src, n);
        return off;
    };
    for (BatchGroup& G : P->groups) {
        const size_t nseq = recs[G.slots[0]].size();
        G.seq.resize(nseq);
        for (size_t i = 0; i < nseq; ++i) {
            BatchPos& bp = G.seq[i];
            const LaunchRecord& l0 = recs[G.slots[0]][i];
            bp.kind = l0.kind;
            bp.block = l0.block;
            bp.lds = 0;
            bp.ns = (int)G.slots.size();
            std::vector<unsigned char> tab;
            std::vector<unsigned> starts;
            unsigned total = 0;
            for (int q : G.slots) {
                const LaunchRecord& l = recs[q][i];
                starts.push_back(total);
                total += l.grid.x * l.grid.y * l.grid.z;
                bp.block.x = std::max(bp.block.x, l.block.x);
                bp.lds = std::max(bp.lds, l.lds);
                tab.insert(tab.end(), l.rec.begin(), l.rec.end());
            }
            starts.push_back(total);
            bp.total = total;
            bp.tab_off = put(tab.data(), tab.size());
            bp.st_off = put(starts.data(), starts.size() * sizeof(unsigned));
        }
        for (int& q : G.slots) q = active[q];   // back to slot ids
        G.direct = G.slots.size() == 1 || P->slots[G.slots[0]].ctx->g.n >= POOL_DIRECT_CELLS;
    }
    if (host.size() > P->tab_cap) {
        dev_free(P->da, P->tab_dev);
        P->tab_dev = nullptr;
        P->tab_cap = 0;
        P->tab_dev = dev_alloc(P->da, host.size());
        if (!P->tab_dev) return pfail(P, DNSLAB_ENOMEM, "allocation of the batched launch tables failed");
        P->tab_cap = host.size();
    }
    if (!host.empty()) PHIP(P, hipMemcpy(P->tab_dev, host.data(), host.size(), hipMemcpyHostToDevice));
    P->active_ids = active;
    P->dirty = false;
    return DNSLAB_OK;
}

int pool_replay(dnslab_pool* P);

// Capture one pool step (every group's batched launches) into a graph.
int pool_capture(dnslab_pool* P) {
    if (P->gexec) {
        PHIP(P, hipGraphExecDestroy(P->gexec));
        P->gexec = nullptr;
    }
    PHIP(P, hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal));
    const int rc = pool_replay(P);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(P->stream, &g);
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : pfail(P, DNSLAB_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    const hipError_t e2 = hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        P->gexec = nullptr;
        return pfail(P, DNSLAB_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e2));
    }
    return DNSLAB_OK;
}

constexpr int POOL_GROUP_STREAMS = 4;

int pool_streams(dnslab_pool* P) {
    if (!P->gs.empty()) return DNSLAB_OK;
    PHIP(P, hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming));
    for (int i = 0; i < POOL_GROUP_STREAMS; ++i) {
        hipStream_t st;
        hipEvent_t ev;
        PHIP(P, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        P->gs.push_back(st);
        PHIP(P, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        P->gev.push_back(ev);
    }
    return DNSLAB_OK;
}

hipStream_t slot_stream(dnslab_pool* P, int slot) {
    return P->gs.empty() ? P->stream : P->gs[slot % (int)P->gs.size()];
}

// Enqueue the deferred scalar halves of direct scenarios and join every group
// stream back into the pool's stream.
int pool_settle(dnslab_pool* P) {
    for (size_t i = 0; i < P->slots.size(); ++i) {
        PoolSlot& S = P->slots[i];
        if (!S.used || !(S.ctx->tail_pending || S.ctx->join_pending)) continue;
        dnslab_ctx* x = S.ctx;
        x->stream = x->cur = slot_stream(P, (int)i);
        const int rc = x->Lo.esz == 8 ? settle<double>(x) : settle<float>(x);
        x->stream = x->cur = P->stream;
        if (rc) return pfail(P, rc, "settle failed: " + x->err);
    }
    for (size_t i = 0; i < P->gs.size(); ++i) {
        PHIP(P, hipEventRecord(P->gev[i], P->gs[i]));
        PHIP(P, hipStreamWaitEvent(P->stream, P->gev[i], 0));
    }
    return DNSLAB_OK;
}

// One pool step: batched group g on group stream g mod 4, direct scenarios on
// their slot's stream, all forked from and joined back into the pool's stream.
int pool_replay(dnslab_pool* P) {
    char* base = (char*)P->tab_dev;
    const int ngs = (int)P->gs.size();
    if (ngs > 0) {
        PHIP(P, hipEventRecord(P->fork_ev, P->stream));
        for (int i = 0; i < ngs; ++i) PHIP(P, hipStreamWaitEvent(P->gs[i], P->fork_ev, 0));
    }
    for (size_t gi = 0; gi < P->groups.size(); ++gi) {
        const BatchGroup& G = P->groups[gi];
        const hipStream_t st_g = ngs > 0 ? P->gs[gi % ngs] : P->stream;
        if (G.direct) {
            // each scenario's plain step (same kernels, so the same result), on
            // a stream fixed per slot so that a step's deferred scalar half is
            // ordered after it; pool_settle enqueues the last one
            for (int slot : G.slots) {
                dnslab_ctx* x = P->slots[slot].ctx;
                const long long hs = x->host_step;
                x->stream = x->cur = slot_stream(P, slot);
                x->overlap = !P->use_graph;
                const int rc = x->Lo.esz == 8 ? one_step<double>(x) : one_step<float>(x);
                x->stream = x->cur = P->stream;
                x->host_step = hs;   // the pool counts the step
                if (rc) return pfail(P, rc, "step failed: " + x->err);
            }
            continue;
        }
        for (const BatchPos& bp : G.seq) {
            const void* tab = base + bp.tab_off;
            const unsigned* st = (const unsigned*)(base + bp.st_off);
            hipError_t e = is_stencil_kind(bp.kind)
                               ? launch_batched_stencil(bp.kind, tab, st, bp.ns, bp.total, bp.block, bp.lds, st_g)
                               : launch_batched_fft(bp.kind, tab, st, bp.ns, bp.total, bp.block, bp.lds, st_g);
            if (e != hipSuccess) return pfail(P, DNSLAB_EHIP, std::string("batched launch: ") + hipGetErrorString(e));
        }
    }
    for (int i = 0; i < ngs; ++i) {
        PHIP(P, hipEventRecord(P->gev[i], P->gs[i]));
        PHIP(P, hipStreamWaitEvent(P->stream, P->gev[i], 0));
    }
    return DNSLAB_OK;
}

size_t count_near_solid(const uint8_t* beta, int nx, int ny, int nz) {
    size_t cnt = 0;
    for_each_cell_solid_neighbours(beta, nx, ny, nz, [&](size_t, unsigned m) { cnt += m != 0; });
    return cnt;
}

}  // namespace

extern "C" {

int dnslab_pool_create(size_t hbm_budget, int32_t precision, void* stream, void* (*alloc)(size_t, void*),
                       void (*free_)(void*, void*), void* alloc_user, dnslab_pool** out) {
    if (!out) return pfail(nullptr, DNSLAB_EINVAL, "out is NULL");
    if (precision != DNSLAB_FP64 && precision != DNSLAB_FP32_REFINE) return pfail(nullptr, DNSLAB_EINVAL, "bad precision");
    if ((alloc == nullptr) != (free_ == nullptr)) return pfail(nullptr, DNSLAB_EINVAL, "alloc and free_ must both be set or both be NULL");
    try {
        dnslab_pool* P = new dnslab_pool();
        P->budget = hbm_budget;
        P->precision = precision;
        P->da.alloc = alloc;
        P->da.free_ = free_;
        P->da.user = alloc_user;
        P->stream = (hipStream_t)stream;
        if (hipStreamCreateWithFlags(&P->admit_stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            delete P;
            return pfail(nullptr, DNSLAB_EHIP, "creating the admission stream failed");
        }
        *out = P;
        return DNSLAB_OK;
    } catch (...) {
        return pfail(nullptr, DNSLAB_ENOMEM, "host allocation failed");
    }
}

int dnslab_pool_admit(dnslab_pool* P, const dnslab_params* params, int64_t target_steps, const uint8_t* beta_host,
                      int64_t n_forced, const int64_t* fidx_host, const double* fS_host, const double* fuset_host,
                      const double* fcset_host, const uint8_t* room_host, const double* u0, const double* v0,
                      const double* w0, const double* p0, const double* c0, int32_t* slot_out) {
    if (!P) return pfail(nullptr, DNSLAB_EINVAL, "pool is NULL");
    try {
        std::string why;
        int rc = validate(params, why);
        if (rc) return pfail(P, rc, why);
        if (params->precision != P->precision) return pfail(P, DNSLAB_EINVAL, "precision differs from the pool's");
        if (!beta_host || !u0 || !v0 || !w0 || !p0 || !c0 || !slot_out || target_steps < 0)
            return pfail(P, DNSLAB_EINVAL, "bad argument");
        if (n_forced < 0 || (n_forced > 0 && (!fidx_host || !fS_host || !fuset_host || !fcset_host)))
            return pfail(P, DNSLAB_EINVAL, "bad forcing arguments");
        dnslab_params prm = *params;
        prm.stream = P->admit_stream;
        prm.alloc = P->da.alloc;       // the pool's memory, whatever the scenario's params say
        prm.free_ = P->da.free_;
        prm.alloc_user = P->da.user;
        const Layout Lo = make_layout(&prm, (int)n_forced);
        const size_t n = (size_t)Lo.n, esz = Lo.esz;
        const size_t field = align_up(n * esz, 256);
        const size_t nib = count_near_solid(beta_host, prm.nx, prm.ny, prm.nz);
        const size_t bytes = 5 * field + Lo.total + align_up(nib * 4, 256) + align_up(nib, 256) + nib * esz +
                             POOL_TABLE_RESERVE;
        // static inputs go through a device staging buffer (dnslab_init copies
        // them); it is kept between admissions and counted in the budget
        const size_t nf = (size_t)n_forced;
        const size_t tb = align_up(n, 256) + (room_host ? align_up(n, 256) : 0) + nf * (8 + 8 + 24 + 8) + 1024;
        const size_t stage_growth = tb > P->stage_cap ? tb - P->stage_cap : 0;
        if (P->used + bytes + stage_growth > P->budget) return pfail(P, DNSLAB_EAGAIN, "HBM budget exhausted");
        PoolSlot S;
        S.bytes = bytes;
        S.target = target_steps;
        S.state = dev_alloc(P->da, 5 * field);
        if (!S.state) return pfail(P, DNSLAB_ENOMEM, "allocation of the scenario state failed");
        // upload the initial fields in the field type
        std::vector<unsigned char> tmp(n * esz);
        const double* src[5] = {u0, v0, w0, p0, c0};
        void* dst[5];
        for (int f = 0; f < 5; ++f) {
            dst[f] = (char*)S.state + f * field;
            if (esz == 8) std::memcpy(tmp.data(), src[f], n * 8);
            else
                for (size_t i = 0; i < n; ++i) ((float*)tmp.data())[i] = (float)src[f][i];
            if (hipMemcpy(dst[f], tmp.data(), n * esz, hipMemcpyHostToDevice) != hipSuccess) {
                dev_free(P->da, S.state);
                return pfail(P, DNSLAB_EHIP, "uploading initial fields failed");
            }
        }
        if (tb > P->stage_cap) {
            dev_free(P->da, P->stage);
            P->used -= P->stage_cap;
            P->stage = nullptr;
            P->stage_cap = 0;
            P->stage = dev_alloc(P->da, tb);
            if (!P->stage) {
                dev_free(P->da, S.state);
                return pfail(P, DNSLAB_ENOMEM, "staging allocation failed");
            }
            P->stage_cap = tb;
            P->used += tb;
        }
        char* t = (char*)P->stage;
        uint8_t* beta_d = (uint8_t*)t;
        t += align_up(n, 256);
        uint8_t* room_d = nullptr;
        if (room_host) { room_d = (uint8_t*)t; t += align_up(n, 256); }
        int64_t* fidx_d = (int64_t*)t; t += nf * 8;
        double* fS_d = (double*)t; t += nf * 8;
        double* fus_d = (double*)t; t += nf * 24;
        double* fcs_d = (double*)t;
        bool ok = hipMemcpy(beta_d, beta_host, n, hipMemcpyHostToDevice) == hipSuccess;
        if (room_host) ok = ok && hipMemcpy(room_d, room_host, n, hipMemcpyHostToDevice) == hipSuccess;
        if (nf) {
            ok = ok && hipMemcpy(fidx_d, fidx_host, nf * 8, hipMemcpyHostToDevice) == hipSuccess;
            ok = ok && hipMemcpy(fS_d, fS_host, nf * 8, hipMemcpyHostToDevice) == hipSuccess;
            ok = ok && hipMemcpy(fus_d, fuset_host, nf * 24, hipMemcpyHostToDevice) == hipSuccess;
            ok = ok && hipMemcpy(fcs_d, fcset_host, nf * 8, hipMemcpyHostToDevice) == hipSuccess;
        }
        if (!ok) {
            dev_free(P->da, S.state);
            return pfail(P, DNSLAB_EHIP, "uploading inputs failed");
        }
        rc = dnslab_init(&prm, beta_d, n_forced, nf ? fidx_d : nullptr, nf ? fS_d : nullptr, nf ? fus_d : nullptr,
                         nf ? fcs_d : nullptr, room_d, dst[0], dst[1], dst[2], dst[3], dst[4], &S.ctx);
        if (rc) {
            dev_free(P->da, S.state);
            return pfail(P, rc, std::string("init: ") + dnslab_last_error(nullptr));
        }
        // dnslab_init has completed its work on the admission stream; from now on
        // the scenario is advanced on the pool's stream.
        S.ctx->stream = P->stream;
        S.ctx->cur = P->stream;
        S.ctx->P.stream = P->stream;
        S.ctx->overlap = false;   // the pool replays whole recorded steps on its one stream
        S.used = true;
        int slot = -1;
        for (size_t i = 0; i < P->slots.size(); ++i)
            if (!P->slots[i].used) { slot = (int)i; break; }
        if (slot < 0) {
            slot = (int)P->slots.size();
            P->slots.push_back(S);
        } else {
            P->slots[slot] = S;
        }
        P->used += bytes;
        P->dirty = true;
        *slot_out = slot;
        return DNSLAB_OK;
    } catch (...) {
        return pfail(P, DNSLAB_ENOMEM, "host allocation failed");
    }
}

int dnslab_pool_step(dnslab_pool* P, int32_t nsteps) {
    if (!P) return pfail(nullptr, DNSLAB_EINVAL, "pool is NULL");
    if (nsteps < 0) return pfail(P, DNSLAB_EINVAL, "nsteps < 0");
    try {
        for (int it = 0; it < nsteps; ++it) {
            std::vector<int> active;
            for (size_t i = 0; i < P->slots.size(); ++i)
                if (P->slots[i].used && P->slots[i].done < P->slots[i].target) active.push_back((int)i);
            if (active.empty()) break;
            if (P->dirty || active != P->active_ids) {
                int rc = pool_streams(P);
                if (!rc) rc = pool_settle(P);
                if (!rc) rc = pool_rebuild(P, active);
                if (!rc && P->use_graph) rc = pool_capture(P);
                if (rc) return rc;
            }
            if (P->use_graph) {
                PHIP(P, hipGraphLaunch(P->gexec, P->stream));
            } else {
                int rc = pool_replay(P);
                if (rc) return rc;
            }
            for (int i : active) {
                P->slots[i].done += 1;
                P->slots[i].ctx->host_step += 1;
            }
        }
        return pool_settle(P);
    } catch (...) {
        return pfail(P, DNSLAB_ENOMEM, "host allocation failed");
    }
}

int dnslab_pool_query(dnslab_pool* P, int32_t slot, dnslab_diag* last, int64_t* steps_done, int32_t* done) {
    if (!P) return pfail(nullptr, DNSLAB_EINVAL, "pool is NULL");
    if (slot < 0 || slot >= (int)P->slots.size() || !P->slots[slot].used) return pfail(P, DNSLAB_EINVAL, "bad slot");
    PoolSlot& S = P->slots[slot];
    if (steps_done) *steps_done = S.done;
    if (done) *done = S.done >= S.target ? 1 : 0;
    if (last) {
        if (S.done == 0) {
            std::memset(last, 0, sizeof(*last));
        } else {
            const int rc = dnslab_read_diags(S.ctx, 1, last);
            if (rc) return pfail(P, rc, S.ctx->err);
        }
    }
    return DNSLAB_OK;
}

int dnslab_pool_read_field(dnslab_pool* P, int32_t slot, int32_t field, double* host_out) {
    if (!P) return pfail(nullptr, DNSLAB_EINVAL, "pool is NULL");
    if (slot < 0 || slot >= (int)P->slots.size() || !P->slots[slot].used || field < 0 || field > 4 || !host_out)
        return pfail(P, DNSLAB_EINVAL, "bad argument");
    dnslab_ctx* x = P->slots[slot].ctx;
    const size_t n = (size_t)x->g.n, esz = x->Lo.esz;
    void* f[5] = {x->u, x->v, x->w, x->p, x->c};
    PHIP(P, hipStreamSynchronize(P->stream));
    if (esz == 8) {
        PHIP(P, hipMemcpy(host_out, f[field], n * 8, hipMemcpyDeviceToHost));
    } else {
        try {
            std::vector<float> tmp(n);
            PHIP(P, hipMemcpy(tmp.data(), f[field], n * 4, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < n; ++i) host_out[i] = tmp[i];
        } catch (...) {
            return pfail(P, DNSLAB_ENOMEM, "host allocation failed");
        }
    }
    return DNSLAB_OK;
}

int dnslab_pool_release(dnslab_pool* P, int32_t slot) {
    if (!P) return pfail(nullptr, DNSLAB_EINVAL, "pool is NULL");
    if (slot < 0 || slot >= (int)P->slots.size() || !P->slots[slot].used) return pfail(P, DNSLAB_EINVAL, "bad slot");
    PoolSlot& S = P->slots[slot];
    dnslab_destroy(S.ctx);      // synchronises the stream
    dev_free(P->da, S.state);
    P->used -= S.bytes;
    S = PoolSlot();
    P->dirty = true;
    return DNSLAB_OK;
}

int dnslab_pool_usage(dnslab_pool* P, size_t* bytes_in_use, int32_t* active, int32_t* resident) {
    if (!P) return pfail(nullptr, DNSLAB_EINVAL, "pool is NULL");
    int a = 0, r = 0;
    for (const PoolSlot& S : P->slots)
        if (S.used) {
            ++r;
            if (S.done < S.target) ++a;
        }
    if (bytes_in_use) *bytes_in_use = P->used;
    if (active) *active = a;
    if (resident) *resident = r;
    return DNSLAB_OK;
}

int dnslab_pool_set_graph(dnslab_pool* P, int32_t enable) {
    if (!P) return pfail(nullptr, DNSLAB_EINVAL, "pool is NULL");
    if (enable != 0 && enable != 1) return pfail(P, DNSLAB_EINVAL, "enable must be 0 or 1");
    if (enable && !P->stream) return pfail(P, DNSLAB_EINVAL, "graph replay needs a non-NULL stream");
    P->use_graph = enable != 0;
    P->dirty = true;
    return DNSLAB_OK;
}

const char* dnslab_pool_last_error(const dnslab_pool* P) { return P ? P->err.c_str() : g_thread_err.c_str(); }

void dnslab_pool_destroy(dnslab_pool* P) {
    if (!P) return;
    (void)hipStreamSynchronize(P->stream);
    for (size_t i = 0; i < P->slots.size(); ++i)
        if (P->slots[i].used) dnslab_pool_release(P, (int)i);
    if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
    for (hipStream_t st : P->gs) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (hipEvent_t ev : P->gev) (void)hipEventDestroy(ev);
    if (P->fork_ev) (void)hipEventDestroy(P->fork_ev);
    dev_free(P->da, P->tab_dev);
    if (P->admit_stream) (void)hipStreamDestroy(P->admit_stream);
    dev_free(P->da, P->stage);
    delete P;
}

}  // extern "C"
