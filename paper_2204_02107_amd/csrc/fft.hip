// FFT Poisson solve of Section 2.2 on gfx950.
//
// The pressure equation is diagonal in Fourier space.  Each iteration of the
// immersed-boundary loop is five passes over HBM:
//   x-forward  : r = r0 + div((1-beta) grad p) at flagged cells, real-to-complex
//                along x via a half-length complex FFT and the even/odd split;
//   y-forward  : complex FFT along y;
//   z-solve    : complex FFT along z, multiply by 1/(lambda N), inverse FFT
//                along z, all in LDS (one read and one write of the spectrum);
//   y-inverse  : complex inverse FFT along y;
//   x-inverse  : complex-to-real along x into p.
// Every pass stages whole lines in LDS and runs a self-sorting Stockham FFT
// there (mixed radix 8/4/2/3), so each pass touches HBM once for reading and
// once for writing.  Strided y/z lines are loaded as tiles of TX consecutive
// kx columns (TX complex values contiguous per row) to keep the accesses
// coalesced.  Grids with small (ky, kz) planes instead store the spectrum
// plane by plane and run y-forward, z-solve and y-inverse as one fused pass
// with one block per kx plane.
#include "fft.h"

#include <algorithm>

// Column passes: the last radix pass stores to the spectrum (plain and
// batched kernels alike, so that both give the same results).  On
// 1024x512x256 the FP32 y pass went from 259 to 214 us, the z solve from 372
// to 343 us (FP32) and from 549 to 509 us (FP64), the FP64 y pass unchanged;
// 512x256x192 FP64 y 72 -> 68 us, z 108 -> 91 us.
#ifndef DNSLAB_COL_DIRECT
#define DNSLAB_COL_DIRECT 1
#endif
// Listed cells per thread of the IB right-hand side.  Issuing all of a
// cell's gathers of p before the sums (instead of one gather per branch of
// the sum) took the kernel on 1024x512x256 from 102 to 89 us (FP64) and from
// 85 to 68 us (FP32); 4 or 8 cells per thread gained nothing more (8: 97 us).
#ifndef DNSLAB_IB_CPT
#define DNSLAB_IB_CPT 1
#endif
constexpr int IB_CPT = DNSLAB_IB_CPT;
#ifndef DNSLAB_COL_XCD
#define DNSLAB_COL_XCD 1       // column passes: XCD-aware tile order (xcd_tile)
#endif
#ifndef DNSLAB_FFT_TPL_MUL
#define DNSLAB_FFT_TPL_MUL 1   // threads per line = MUL * n / rad[0] (extra threads only stage memory)
#endif


namespace dnslab {

namespace {

template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ C2<T> cmulc(C2<T> a, C2<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ C2<T> conj_(C2<T> a) { return {a.x, -a.y}; }
// multiply by -i (forward sign) or +i (inverse sign)
template <typename T, bool INV>
__device__ __forceinline__ C2<T> rot(C2<T> a) {
    return INV ? C2<T>{-a.y, a.x} : C2<T>{a.y, -a.x};
}

// In-register DFT of length R with kernel e^{-+2 pi i r m / R}.
template <typename T, int R, bool INV>
struct DFT;

template <typename T, bool INV>
struct DFT<T, 2, INV> {
    static __device__ __forceinline__ void run(C2<T>* v) {
        const C2<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <typename T, bool INV>
struct DFT<T, 4, INV> {
    static __device__ __forceinline__ void run(C2<T>* v) {
        const C2<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        const C2<T> t2 = cadd(v[1], v[3]), t3 = rot<T, INV>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

template <typename T, bool INV>
struct DFT<T, 8, INV> {
    static __device__ __forceinline__ void run(C2<T>* v) {
        C2<T> e[4] = {v[0], v[2], v[4], v[6]};
        C2<T> o[4] = {v[1], v[3], v[5], v[7]};
        DFT<T, 4, INV>::run(e);
        DFT<T, 4, INV>::run(o);
        const T h = T(0.70710678118654752440);
        // o[m] *= w8^m, w8 = e^{-+ i pi / 4}
        const C2<T> o1 = INV ? C2<T>{h * (o[1].x - o[1].y), h * (o[1].x + o[1].y)}
                             : C2<T>{h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};
        const C2<T> o2 = rot<T, INV>(o[2]);
        const C2<T> o3 = INV ? C2<T>{-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y)}
                             : C2<T>{h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
};

template <typename T, bool INV>
struct DFT<T, 3, INV> {
    static __device__ __forceinline__ void run(C2<T>* v) {
        const T h = T(0.86602540378443864676);   // sqrt(3)/2
        const C2<T> t = cadd(v[1], v[2]);
        const C2<T> sd = rot<T, INV>(csub(v[1], v[2]));
        const C2<T> m = {v[0].x - T(0.5) * t.x, v[0].y - T(0.5) * t.y};
        v[0] = cadd(v[0], t);
        v[1] = {m.x + h * sd.x, m.y + h * sd.y};
        v[2] = {m.x - h * sd.x, m.y - h * sd.y};
    }
};

// One Stockham pass of radix R over all lines held in LDS.  Element e of line
// l lives at s[l*ls + e*es].  Butterfly b belongs to line b & (nl-1), so
// consecutive threads work on consecutive lines.  In place: every thread
// reads its inputs, the block synchronises, then writes the outputs.
template <typename T, int R, int MAXB, bool INV>
__device__ __forceinline__ void stockham_pass(C2<T>* s, int n, int ns, const C2<T>* W, int es,
                                              int ls, int lg_nl, int tid, int nthr) {
    const int nbl = n / R;
    const int nb = nbl << lg_nl;
    const int mask = (1 << lg_nl) - 1;
    C2<T> v[MAXB][R];
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int b = tid + q * nthr;
        if (b < nb) {
            const int j = b >> lg_nl;
            const C2<T>* base = s + (b & mask) * ls;
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = base[(j + r * nbl) * es];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int b = tid + q * nthr;
        if (b < nb) {
            const int j = b >> lg_nl;
            const int k = j % ns;
            if (ns > 1) {
                const int step = n / (ns * R);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const C2<T> w = W[r * k * step];
                    v[q][r] = INV ? cmulc(v[q][r], w) : cmul(v[q][r], w);
                }
            }
            DFT<T, R, INV>::run(v[q]);
            C2<T>* base = s + (b & mask) * ls;
            const int d = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) base[(d + r * ns) * es] = v[q][r];
        }
    }
    __syncthreads();
}

template <typename T, bool INV>
__device__ void fft_lds_runtime(C2<T>* s, const AxisPlan& ap, const C2<T>* W, int es, int ls, int lg_nl, int tid,
                                int nthr) {
    int ns = 1;
    for (int p = 0; p < ap.npass; ++p) {
        const int R = ap.rad[p];
        if (R == 8) stockham_pass<T, 8, 1, INV>(s, ap.n, ns, W, es, ls, lg_nl, tid, nthr);
        else if (R == 4) stockham_pass<T, 4, 2, INV>(s, ap.n, ns, W, es, ls, lg_nl, tid, nthr);
        else if (R == 2) stockham_pass<T, 2, 4, INV>(s, ap.n, ns, W, es, ls, lg_nl, tid, nthr);
        else stockham_pass<T, 3, 3, INV>(s, ap.n, ns, W, es, ls, lg_nl, tid, nthr);
        ns *= R;
    }
}

// Compile-time plan: the same radix sequence as make_axis_plan (8s first,
// then 4/2, then 3s), so that the threads per line match the launch.
struct CPlan {
    int np;
    int r[FFT_MAX_PASSES];
};
constexpr CPlan cplan(int n) {
    CPlan p{0, {}};
    int a = 0, b = 0, m = n;
    while (m > 1 && m % 2 == 0) { m /= 2; ++a; }
    while (m > 1 && m % 3 == 0) { m /= 3; ++b; }
    const int eights = a / 3, rest = a % 3;
    if (rest == 1 && eights >= 1) {
        for (int i = 0; i < eights - 1; ++i) p.r[p.np++] = 8;
        p.r[p.np++] = 4;
        p.r[p.np++] = 4;
    } else {
        for (int i = 0; i < eights; ++i) p.r[p.np++] = 8;
        if (rest == 2) p.r[p.np++] = 4;
        if (rest == 1) p.r[p.np++] = 2;
    }
    for (int i = 0; i < b; ++i) p.r[p.np++] = 3;
    return p;
}
constexpr int cns(int n, int pass) {
    const CPlan p = cplan(n);
    int ns = 1;
    for (int i = 0; i < pass; ++i) ns *= p.r[i];
    return ns;
}

// One Stockham pass with the transform length, radix and span known at
// compile time (the index arithmetic becomes shifts and constant multiplies).
// Barrier between LDS phases of one block.  The plain one (__syncthreads)
// also waits for the wave's outstanding global memory operations; the LDS
// one waits only for its LDS operations, so that asynchronous global -> LDS
// loads of another buffer stay in flight across it.
template <bool LB>
__device__ __forceinline__ void phase_barrier() {
    if (LB) asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else __syncthreads();
}

// Epilogue of a pass: out value for line (column) c, row i.
struct NoEpi {
    template <typename V>
    __device__ __forceinline__ V operator()(int, int, V v) const { return v; }
};

template <typename T, int R, int MAXB, bool INV, int N, int NS, bool LB = false, class Epi = NoEpi>
__device__ __forceinline__ void stockham_pass_c(C2<T>* s, const C2<T>* W, int es, int ls, int lg_nl, int tid,
                                                int nthr, Epi epi = Epi()) {
    constexpr int nbl = N / R;
    constexpr int step = N / (NS * R);
    const int nb = nbl << lg_nl;
    const int mask = (1 << lg_nl) - 1;
    C2<T> v[MAXB][R];
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int b = tid + q * nthr;
        if (b < nb) {
            const int j = b >> lg_nl;
            const C2<T>* base = s + (b & mask) * ls;
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = base[(j + r * nbl) * es];
        }
    }
    phase_barrier<LB>();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int b = tid + q * nthr;
        if (b < nb) {
            const int j = b >> lg_nl;
            const int k = j % NS;
            if (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const C2<T> w = W[r * k * step];
                    v[q][r] = INV ? cmulc(v[q][r], w) : cmul(v[q][r], w);
                }
            }
            DFT<T, R, INV>::run(v[q]);
            C2<T>* base = s + (b & mask) * ls;
            const int d = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) base[(d + r * NS) * es] = epi(b & mask, d + r * NS, v[q][r]);
        }
    }
    phase_barrier<LB>();
}

// The last pass of a chain with its outputs handed to out(line, row, value)
// instead of written back in place: no LDS writes, hence no barrier.
template <typename T, int R, int MAXB, bool INV, int N, int NS, class Out>
__device__ __forceinline__ void stockham_pass_out(const C2<T>* s, const C2<T>* W, int es, int ls, int lg_nl, int tid,
                                                  int nthr, Out out) {
    constexpr int nbl = N / R;
    constexpr int step = N / (NS * R);
    const int nb = nbl << lg_nl;
    const int mask = (1 << lg_nl) - 1;
    C2<T> v[MAXB][R];
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int b = tid + q * nthr;
        if (b < nb) {
            const int j = b >> lg_nl;
            const C2<T>* base = s + (b & mask) * ls;
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = base[(j + r * nbl) * es];
        }
    }
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int b = tid + q * nthr;
        if (b < nb) {
            const int j = b >> lg_nl;
            const int k = j % NS;
            if (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const C2<T> w = W[r * k * step];
                    v[q][r] = INV ? cmulc(v[q][r], w) : cmul(v[q][r], w);
                }
            }
            DFT<T, R, INV>::run(v[q]);
            const int d = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) out(b & mask, d + r * NS, v[q][r]);
        }
    }
}

template <typename T, bool INV, int N, int P, bool LB = false>
__device__ __forceinline__ void fft_chain(C2<T>* s, const C2<T>* W, int es, int ls, int lg_nl, int tid, int nthr) {
    constexpr CPlan pl = cplan(N);
    if constexpr (P < pl.np) {
        constexpr int R = pl.r[P];
        constexpr int MAXB = (pl.r[0] + R - 1) / R;
        stockham_pass_c<T, R, MAXB, INV, N, cns(N, P), LB>(s, W, es, ls, lg_nl, tid, nthr);
        fft_chain<T, INV, N, P + 1, LB>(s, W, es, ls, lg_nl, tid, nthr);
    }
}

// The chain of compile-time passes with a different last pass: OUT, its
// outputs go to f(line, row, value) (no LDS writes); otherwise written back in
// place through the epilogue f.
template <typename T, bool INV, int N, int P, bool OUT, bool LB = false, class F>
__device__ __forceinline__ void fft_chain_last(C2<T>* s, const C2<T>* W, int es, int ls, int lg_nl, int tid, int nthr,
                                               F f) {
    constexpr CPlan pl = cplan(N);
    constexpr int R = pl.r[P];
    constexpr int MAXB = (pl.r[0] + R - 1) / R;
    if constexpr (P + 1 < pl.np) {
        stockham_pass_c<T, R, MAXB, INV, N, cns(N, P), LB>(s, W, es, ls, lg_nl, tid, nthr);
        fft_chain_last<T, INV, N, P + 1, OUT, LB>(s, W, es, ls, lg_nl, tid, nthr, f);
    } else if constexpr (OUT) {
        stockham_pass_out<T, R, MAXB, INV, N, cns(N, P)>(s, W, es, ls, lg_nl, tid, nthr, f);
    } else {
        stockham_pass_c<T, R, MAXB, INV, N, cns(N, P), LB>(s, W, es, ls, lg_nl, tid, nthr, f);
    }
}

// In-place transform of all lines held in LDS; specialised chains for the
// common lengths, the runtime plan otherwise.
// Inlined form for kernels that keep data in registers across the transform
// (a call would spill them around it).
template <typename T, bool INV>
__device__ __forceinline__ void fft_lds_inl(C2<T>* s, const AxisPlan& ap, const C2<T>* W, int es, int ls, int lg_nl,
                                            int tid, int nthr) {
    switch (ap.n) {
        case 1: return;
        case 16: fft_chain<T, INV, 16, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 32: fft_chain<T, INV, 32, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 48: fft_chain<T, INV, 48, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 64: fft_chain<T, INV, 64, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 96: fft_chain<T, INV, 96, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 128: fft_chain<T, INV, 128, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        default: {
            int ns = 1;
            for (int p = 0; p < ap.npass; ++p) {
                const int R = ap.rad[p];
                if (R == 8) stockham_pass<T, 8, 1, INV>(s, ap.n, ns, W, es, ls, lg_nl, tid, nthr);
                else if (R == 4) stockham_pass<T, 4, 2, INV>(s, ap.n, ns, W, es, ls, lg_nl, tid, nthr);
                else if (R == 2) stockham_pass<T, 2, 4, INV>(s, ap.n, ns, W, es, ls, lg_nl, tid, nthr);
                else stockham_pass<T, 3, 3, INV>(s, ap.n, ns, W, es, ls, lg_nl, tid, nthr);
                ns *= R;
            }
            return;
        }
    }
}

template <typename T, bool INV>
__device__ void fft_lds(C2<T>* s, const AxisPlan& ap, const C2<T>* W, int es, int ls, int lg_nl, int tid, int nthr) {
    switch (ap.n) {
        case 1: return;
        case 16: fft_chain<T, INV, 16, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 32: fft_chain<T, INV, 32, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 48: fft_chain<T, INV, 48, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 64: fft_chain<T, INV, 64, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 96: fft_chain<T, INV, 96, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 128: fft_chain<T, INV, 128, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 192: fft_chain<T, INV, 192, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 256: fft_chain<T, INV, 256, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 384: fft_chain<T, INV, 384, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 512: fft_chain<T, INV, 512, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 768: fft_chain<T, INV, 768, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        case 1024: fft_chain<T, INV, 1024, 0>(s, W, es, ls, lg_nl, tid, nthr); return;
        default: fft_lds_runtime<T, INV>(s, ap, W, es, ls, lg_nl, tid, nthr); return;
    }
}

// Immersed-boundary right-hand side at the listed cells (Section 2.2):
// r = r0 + sum_a [ (1-beta)(x+e_a) D_a p(x+e_a) - (1-beta)(x-e_a) D_a p(x-e_a) ] / (2 dx_a)
// with central D_a; (1-beta) is 1 exactly where the mask bit says "solid".
template <typename T>
__device__ __forceinline__ void ib_rhs_body(const IbArgs<T>& A, unsigned blk) {
    // IB_CPT listed cells per thread (entries blk * blockDim.x * IB_CPT + q *
    // blockDim.x + tid): the list loads of all of them, then all their
    // gathers of p, then the sums, so that a thread's gathers are in flight
    // together.
    const IBList& ib = A.ib;
    const Grid& g = A.g;
    const T* __restrict__ p = A.p;
    T* __restrict__ r = A.r;
    T* __restrict__ r0s = A.r0s;
    const int first = A.first;
    const int e0 = (int)(blk * blockDim.x) * IB_CPT + (int)threadIdx.x;
    const unsigned nx = g.nx, ny = g.ny, nz = g.nz;
    const unsigned nxy = nx * ny;
    unsigned idx[IB_CPT], mask[IB_CPT];
#pragma unroll
    for (int q = 0; q < IB_CPT; ++q) {
        const int e = e0 + q * (int)blockDim.x;
        idx[q] = 0;
        mask[q] = 0;
        if (e < ib.n) {
            idx[q] = (unsigned)ib.idx[e];
            mask[q] = ib.mask[e];
        }
    }
    T r0[IB_CPT], p0[IB_CPT], pn[IB_CPT][6];
#pragma unroll
    for (int q = 0; q < IB_CPT; ++q) {
        const int e = e0 + q * (int)blockDim.x;
        const bool live = e < ib.n;
        const unsigned id = idx[q], mk = mask[q];
        const unsigned i = id % nx, jk = id / nx;
        const unsigned j = jk % ny, k = jk / ny;
        // +-2 neighbours along each axis with periodic wrap
        const unsigned nb[6] = {id - i + (i + 2) % nx, id - i + (i + 2 * nx - 2) % nx,
                                id + (((j + 2) % ny) - j) * nx, id + (((j + 2 * ny - 2) % ny) - j) * nx,
                                id + (((k + 2) % nz) - k) * nxy, id + (((k + 2 * nz - 2) % nz) - k) * nxy};
        r0[q] = T(0);
        p0[q] = T(0);
        if (live) {
            r0[q] = first ? r[id] : r0s[e];
            p0[q] = p[id];
        }
#pragma unroll
        for (int d = 0; d < 6; ++d) pn[q][d] = (live && (mk >> d & 1u)) ? p[nb[d]] : T(0);
    }
    const T hx = T(g.inv2d[0]), hy = T(g.inv2d[1]), hz = T(g.inv2d[2]);
#pragma unroll
    for (int q = 0; q < IB_CPT; ++q) {
        const int e = e0 + q * (int)blockDim.x;
        if (e >= ib.n) continue;
        const unsigned mk = mask[q];
        const T c = p0[q];
        T acc = T(0);
        if (mk & 1u) acc += ((pn[q][0] - c) * hx) * hx;
        if (mk & 2u) acc -= ((c - pn[q][1]) * hx) * hx;
        if (mk & 4u) acc += ((pn[q][2] - c) * hy) * hy;
        if (mk & 8u) acc -= ((c - pn[q][3]) * hy) * hy;
        if (mk & 16u) acc += ((pn[q][4] - c) * hz) * hz;
        if (mk & 32u) acc -= ((c - pn[q][5]) * hz) * hz;
        if (first) r0s[e] = r0[q];
        r[idx[q]] = r0[q] + acc;
    }
}

// X[k] of the real transform from Z = FFT(x_even + i x_odd):
// E = (Z[k] + conj Z[m-k])/2, O = -i (Z[k] - conj Z[m-k])/2, X[k] = E + w^k O.
template <typename T>
__device__ __forceinline__ C2<T> r2c_post(C2<T> za, C2<T> zb, C2<T> w) {
    const C2<T> zc = conj_(zb);
    const C2<T> e = cscale(cadd(za, zc), T(0.5));
    const C2<T> o = cscale(rot<T, false>(csub(za, zc)), T(0.5));
    return cadd(e, cmul(w, o));
}
// Z[k] for the inverse from X[k], X[m-k] (unnormalised: twice the even/odd
// spectra): E = X[k] + conj X[m-k], O = (X[k] - conj X[m-k]) conj(w^k), Z = E + i O.
template <typename T>
__device__ __forceinline__ C2<T> c2r_pre(C2<T> xa, C2<T> xb, C2<T> w) {
    const C2<T> xc = conj_(xb);
    const C2<T> e = cadd(xa, xc);
    const C2<T> o = cmulc(csub(xa, xc), w);
    return cadd(e, rot<T, true>(o));
}

// Batched global -> register -> LDS staging: every thread issues all of its
// loads before the first LDS store, so that a block keeps many independent
// memory requests in flight (the passes are otherwise latency bound).
constexpr int STAGE_MAX = 9;   // elements per thread: at most rad[0] (+1 for the x inverse)

// Split e into (line, element) for line length m (power of two: shifts).
struct LineSplit {
    int m, lgm;
    __device__ __forceinline__ void split(int e, int& l, int& n) const {
        if (lgm >= 0) { l = e >> lgm; n = e & (m - 1); }
        else { l = e / m; n = e - l * m; }
    }
};
__device__ __forceinline__ LineSplit line_split(int m) {
    LineSplit ls;
    ls.m = m;
    ls.lgm = (m & (m - 1)) == 0 ? __ffs(m) - 1 : -1;
    return ls;
}

template <typename T>
__device__ __forceinline__ void fft_x_fwd_body(const FxfArgs<T>& A, unsigned blk) {
    const FFTArgs<T>& a = A.f;
    const T* __restrict__ r = A.r;
    extern __shared__ unsigned char smem_raw[];
    C2<T>* s = reinterpret_cast<C2<T>*>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lg = a.nl_x, m = a.m, ls = a.ls_x;
    const int line0 = (int)blk << lg;
    const int nlines = a.g.ny * a.g.nz;
    const unsigned nx = a.g.nx;
    const LineSplit sp = line_split(m);
    const int tot = m << lg;
    // the W_m table and the real-transform twist: staged in LDS, or read
    // through the caches (long lines: LDS then holds only the lines)
    const C2<T>* wl = a.wx;
    const C2<T>* tl = a.tw;
    if (a.xtw_lds) {
        C2<T>* w = s + (ls << lg);
        for (int j = tid; j < m; j += nthr) w[j] = a.wx[j];
        for (int j = tid; j <= m; j += nthr) w[m + j] = a.tw[j];
        wl = w;
        tl = w + m;
    }
    C2<T> buf[STAGE_MAX];
#pragma unroll
    for (int q = 0; q < STAGE_MAX; ++q) {
        const int e = tid + q * nthr;
        int l, n;
        sp.split(e, l, n);
        buf[q] = C2<T>{T(0), T(0)};
        if (e < tot && line0 + l < nlines)
            buf[q] = *reinterpret_cast<const C2<T>*>(r + (unsigned)(line0 + l) * nx + 2u * (unsigned)n);
    }
#pragma unroll
    for (int q = 0; q < STAGE_MAX; ++q) {
        const int e = tid + q * nthr;
        int l, n;
        sp.split(e, l, n);
        if (e < tot) s[l * ls + n] = buf[q];
    }
    __syncthreads();
    fft_lds<T, false>(s, a.px, wl, 1, ls, lg, tid, nthr);
    const int half = m / 2 + 1;
    // row-major: consecutive threads take consecutive kx of a line; plane-major:
    // consecutive lines of one kx (contiguous there)
    const bool pm = a.ps > 0;
    const size_t ks = pm ? (size_t)a.ps : 1, lstr = pm ? 1 : (size_t)a.sx;
    for (int e = tid; e < (half << lg); e += nthr) {
        int l, k;
        if (pm) { l = e & ((1 << lg) - 1); k = e >> lg; }
        else { l = e / half; k = e - l * half; }
        const int L = line0 + l;
        if (L >= nlines) continue;
        const C2<T>* zl = s + l * ls;
        C2<T>* out = a.spec + (size_t)L * lstr;
        const C2<T> za = zl[k];
        const C2<T> zb = zl[k == 0 ? 0 : m - k];
        out[k * ks] = r2c_post(za, zb, tl[k]);
        if (m - k != k) out[(m - k) * ks] = r2c_post(zb, za, tl[m - k]);
    }
}

template <typename T>
__device__ __forceinline__ void fft_x_inv_body(const FxiArgs<T>& A, unsigned blk) {
    const FFTArgs<T>& a = A.f;
    T* __restrict__ p = A.p;
    extern __shared__ unsigned char smem_raw[];
    C2<T>* s = reinterpret_cast<C2<T>*>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lg = a.nl_x, m = a.m, ls = a.ls_x;
    const int line0 = (int)blk << lg;
    const int nlines = a.g.ny * a.g.nz;
    const unsigned nx = a.g.nx;
    const C2<T>* wl = a.wx;
    const C2<T>* tl = a.tw;
    if (a.xtw_lds) {
        C2<T>* w = s + (ls << lg);
        for (int j = tid; j < m; j += nthr) w[j] = a.wx[j];
        for (int j = tid; j <= m; j += nthr) w[m + j] = a.tw[j];
        wl = w;
        tl = w + m;
    }
    {
        // Each thread takes (X[k], X[m-k]) pairs of a line straight from the
        // spectrum and stores the twisted pair (Z[k], Z[m-k]) into LDS, so the
        // spectrum is staged once (staging it as is and twisting it in place
        // took one more LDS pass and barrier: 1024x512x256 x inverse 481 ->
        // 453 us FP64, 290 -> 262 us FP32).  Pair e -> (line l, k < m/2 + 1): k fastest
        // for the row-major spectrum, line fastest for the plane-major one
        // (contiguous in either).
        const int half = m / 2 + 1;
        const int tot = half << lg;
        const bool pm = a.ps > 0;
        const size_t ks = pm ? (size_t)a.ps : 1, lstr = pm ? 1 : (size_t)a.sx;
        auto split = [&](int e, int& l, int& k) {
            if (pm) { l = e & ((1 << lg) - 1); k = e >> lg; }
            else { l = e / half; k = e - l * half; }
        };
        auto twist = [&](int l, int k, C2<T> xa, C2<T> xb) {
            C2<T>* zl = s + l * ls;
            if (k == 0) { xa.y = T(0); xb.y = T(0); }   // the real transform ignores Im X[0], Im X[m]
            const C2<T> za = c2r_pre(xa, xb, tl[k]);
            if (k != 0 && m - k != k) zl[m - k] = c2r_pre(xb, xa, tl[m - k]);
            zl[k] = za;
        };
        constexpr int PQ = STAGE_MAX / 2 + 1;
        C2<T> ba[PQ], bb[PQ];
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            const int e = tid + q * nthr;
            int l, k;
            split(e, l, k);
            ba[q] = C2<T>{T(0), T(0)};
            bb[q] = C2<T>{T(0), T(0)};
            if (e < tot && line0 + l < nlines) {
                const C2<T>* x = a.spec + (size_t)(line0 + l) * lstr;
                ba[q] = x[k * ks];
                bb[q] = x[(m - k) * ks];
            }
        }
        if (a.xtw_lds) __syncthreads();   // the twist table staged above
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            const int e = tid + q * nthr;
            int l, k;
            split(e, l, k);
            if (e < tot) twist(l, k, ba[q], bb[q]);
        }
        // pairs beyond PQ per thread (only when nthr * PQ < tot)
        for (int e = tid + PQ * nthr; e < tot; e += nthr) {
            int l, k;
            split(e, l, k);
            C2<T> xa = C2<T>{T(0), T(0)}, xb = xa;
            if (line0 + l < nlines) {
                const C2<T>* x = a.spec + (size_t)(line0 + l) * lstr;
                xa = x[k * ks];
                xb = x[(m - k) * ks];
            }
            twist(l, k, xa, xb);
        }
    }
    __syncthreads();
    fft_lds<T, true>(s, a.px, wl, 1, ls, lg, tid, nthr);
    const LineSplit sp = line_split(m);
    for (int e = tid; e < (m << lg); e += nthr) {
        int l, n;
        sp.split(e, l, n);
        const int L = line0 + l;
        if (L < nlines) *reinterpret_cast<C2<T>*>(p + (unsigned)L * nx + 2u * (unsigned)n) = s[l * ls + n];
    }
}

// 1/x to about one ulp: hardware reciprocal refined by two Newton steps.
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// Column passes along y (MODE 0 forward, 1 inverse) or z (MODE 2: forward,
// divide by lambda N with the null modes zeroed, inverse).  A block holds TX
// lines of the spectrum in LDS as [row][line].  Main blocks take TX
// consecutive kx columns 0..m-1 of one plane (TX complex values contiguous
// per row); the Nyquist column kx = m, which would otherwise leave a nearly
// empty tile in every plane, is handled by a few extra blocks that take TX
// different planes of that column each.
// One tile of a column pass: TX consecutive kx columns of one plane (the
// main tiles), or TX planes of the Nyquist column kx = m.
template <typename T>
struct ColTile {
    C2<T>* base;    // element (row, column c) at base[row * rs + c * cs]
    size_t cs;
    int ncol;       // columns present (<= TX)
    int kx0, plane0;
    bool nyq;
};
template <typename T, int MODE>
__device__ __forceinline__ ColTile<T> col_tile(const FFTArgs<T>& a, int b) {
    const bool zp = MODE == 2;
    const int lg = zp ? a.lg_tx_z : a.lg_tx_y, tx = 1 << lg;
    const int ny = a.g.ny, nz = a.g.nz, m = a.m;
    const int nplane = zp ? ny : nz;
    const size_t ps = zp ? (size_t)a.sx : (size_t)ny * a.sx;
    const int ntile = (m + tx - 1) >> lg;
    const int nmain = ntile * nplane;
    ColTile<T> t;
    if (b < nmain) {
        const int tile = b % ntile;
        t.plane0 = b / ntile;
        t.kx0 = tile << lg;
        t.base = a.spec + (size_t)t.plane0 * ps + t.kx0;
        t.cs = 1;
        t.ncol = min(tx, m - t.kx0);
        t.nyq = false;
    } else {
        t.plane0 = (b - nmain) << lg;
        t.kx0 = m;
        t.base = a.spec + (size_t)t.plane0 * ps + m;
        t.cs = ps;
        t.ncol = min(tx, nplane - t.plane0);
        t.nyq = true;
    }
    return t;
}

// The transforms of one staged tile in LDS (s, element (row, c) at
// s[row * TX + c]): y forward or inverse, or z forward, divide, z inverse.
template <typename T, int MODE>
__device__ __forceinline__ void cols_transform(const FFTArgs<T>& a, const ColTile<T>& t, C2<T>* s, const C2<T>* wl,
                                               int tid, int nthr) {
    const int lg = MODE == 2 ? a.lg_tx_z : a.lg_tx_y, tx = 1 << lg;
    if (MODE == 2) {
        const int tot = a.g.nz << lg;
        fft_lds<T, false>(s, a.pz, wl, tx, 1, lg, tid, nthr);
        for (int e = tid; e < tot; e += nthr) {
            const int kz = e >> lg, c = e & (tx - 1);
            if (c < t.ncol) {
                const int kx = t.nyq ? a.m : t.kx0 + c;
                const int ky = t.nyq ? t.plane0 + c : t.plane0;
                const double lam = (a.sz2[kz] + a.sy2[ky]) + a.sx2[kx];   // -lambda
                const T f = lam == 0.0 ? T(0) : T(-a.inv_ntot * recip(lam));
                s[e] = cscale(s[e], f);
            }
        }
        __syncthreads();
        fft_lds<T, true>(s, a.pz, wl, tx, 1, lg, tid, nthr);
    } else {
        fft_lds<T, MODE == 1>(s, a.py, wl, tx, 1, lg, tid, nthr);
    }
}

// The transforms of a staged tile with the last radix pass storing straight
// to the spectrum (each row's TX columns are consecutive lanes, so a wave's
// stores fill whole row segments); the z pass's divide is the epilogue of its
// forward transform's last pass.  Every value gets the same operations as in
// cols_transform and the store loop.
template <typename T, int MODE, int N>
__device__ __forceinline__ void cols_direct(const FFTArgs<T>& a, const ColTile<T>& t, C2<T>* s, const C2<T>* wl,
                                            int tid, int nthr, size_t rs) {
    const int lg = MODE == 2 ? a.lg_tx_z : a.lg_tx_y, tx = 1 << lg;
    // (the functors capture plain values: a reference to the kernel's
    // argument block would put a copy of it on the stack)
    C2<T>* const base = t.base;
    const size_t cs = t.cs;
    const int ncol = t.ncol;
    auto store = [=](int c, int row, const C2<T>& v) {
        if (c < ncol) base[row * rs + c * cs] = v;
    };
    if constexpr (MODE == 2) {
        const double *sx2 = a.sx2, *sy2 = a.sy2, *sz2 = a.sz2;
        const double inv_ntot = a.inv_ntot;
        const int m = a.m, kx0 = t.kx0, plane0 = t.plane0;
        const bool nyq = t.nyq;
        auto divide = [=](int c, int kz, C2<T> v) -> C2<T> {
            if (c < ncol) {
                const int kx = nyq ? m : kx0 + c;
                const int ky = nyq ? plane0 + c : plane0;
                const double lam = (sz2[kz] + sy2[ky]) + sx2[kx];   // -lambda
                const T f = lam == 0.0 ? T(0) : T(-inv_ntot * recip(lam));
                v = cscale(v, f);
            }
            return v;
        };
        fft_chain_last<T, false, N, 0, false>(s, wl, tx, 1, lg, tid, nthr, divide);
        fft_chain_last<T, true, N, 0, true>(s, wl, tx, 1, lg, tid, nthr, store);
    } else {
        fft_chain_last<T, MODE == 1, N, 0, true>(s, wl, tx, 1, lg, tid, nthr, store);
    }
}
// cols_direct for the lengths with a compile-time chain (the ones pipe_length
// lists); false for any other length, with nothing done.
template <typename T, int MODE>
__device__ __forceinline__ bool cols_direct_any(int n, const FFTArgs<T>& a, const ColTile<T>& t, C2<T>* s,
                                                const C2<T>* wl, int tid, int nthr, size_t rs) {
    switch (n) {
        case 64: cols_direct<T, MODE, 64>(a, t, s, wl, tid, nthr, rs); return true;
        case 96: cols_direct<T, MODE, 96>(a, t, s, wl, tid, nthr, rs); return true;
        case 128: cols_direct<T, MODE, 128>(a, t, s, wl, tid, nthr, rs); return true;
        case 192: cols_direct<T, MODE, 192>(a, t, s, wl, tid, nthr, rs); return true;
        case 256: cols_direct<T, MODE, 256>(a, t, s, wl, tid, nthr, rs); return true;
        case 384: cols_direct<T, MODE, 384>(a, t, s, wl, tid, nthr, rs); return true;
        case 512: cols_direct<T, MODE, 512>(a, t, s, wl, tid, nthr, rs); return true;
        case 768: cols_direct<T, MODE, 768>(a, t, s, wl, tid, nthr, rs); return true;
        case 1024: cols_direct<T, MODE, 1024>(a, t, s, wl, tid, nthr, rs); return true;
        default: return false;
    }
}

// DIRECT 1: the transform length has a compile-time chain and the last radix
// pass stores to the spectrum (a kernel of its own for the plain launches: the
// out-of-line runtime transforms beside it would put the argument block, which
// the plain kernels take by value, on the stack); 2: decided per tile (the
// batched kernels, whose scenarios differ in length and whose arguments are
// read in place); 0: transform in place, then store.
template <typename T, int MODE, int DIRECT = 0>
__device__ __forceinline__ void fft_cols_body(const FFTArgs<T>& a, unsigned blk) {
    extern __shared__ unsigned char smem_raw[];
    C2<T>* s = reinterpret_cast<C2<T>*>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const bool zp = MODE == 2;
    const int lg = zp ? a.lg_tx_z : a.lg_tx_y, tx = 1 << lg;
    const int nrow = zp ? a.g.nz : a.g.ny;                 // transform length
    const size_t rs = zp ? (size_t)a.g.ny * a.sx : (size_t)a.sx;   // row (transform) stride
    const ColTile<T> t = col_tile<T, MODE>(a, (int)blk);
    const int tot = nrow << lg;
    C2<T>* wl = s + tot;               // W_nrow table
    {
        const C2<T>* W = zp ? a.wz : a.wy;
        for (int j = tid; j < nrow; j += nthr) wl[j] = W[j];
    }
    {
        C2<T> buf[STAGE_MAX];
#pragma unroll
        for (int q = 0; q < STAGE_MAX; ++q) {
            const int e = tid + q * nthr;
            const int row = e >> lg, c = e & (tx - 1);
            buf[q] = C2<T>{T(0), T(0)};
            if (e < tot && c < t.ncol) buf[q] = t.base[row * rs + c * t.cs];
        }
#pragma unroll
        for (int q = 0; q < STAGE_MAX; ++q) {
            const int e = tid + q * nthr;
            if (e < tot) s[e] = buf[q];
        }
    }
    __syncthreads();
    if constexpr (DIRECT == 1) {
        cols_direct_any<T, MODE>(nrow, a, t, s, wl, tid, nthr, rs);
        return;
    }
    if constexpr (DIRECT == 2 && DNSLAB_COL_DIRECT != 0) {
        if (cols_direct_any<T, MODE>(nrow, a, t, s, wl, tid, nthr, rs)) return;
    }
    cols_transform<T, MODE>(a, t, s, wl, tid, nthr);
#pragma unroll
    for (int q = 0; q < STAGE_MAX; ++q) {
        const int e = tid + q * nthr;
        const int row = e >> lg, c = e & (tx - 1);
        if (e < tot && c < t.ncol) t.base[row * rs + c * t.cs] = s[e];
    }
}

// Column pass over many tiles per block, the next tile's load in flight
// while the current one is transformed: each block walks tiles blockIdx.x,
// + gridDim.x, ... with two LDS tile buffers.  The main tiles are moved
// global -> LDS by the asynchronous LDS loads of gfx950 (16 bytes per lane:
// one FP64 complex, or two adjacent FP32 complex values of a row), which hold
// no registers; the top of each iteration waits for them (vmcnt) and
// synchronises, then issues the next tile's loads before transforming this
// one.  The few Nyquist tiles (strided columns) are loaded the plain way.
// Requires the main tiles' row segments 16-byte aligned and, in FP32, an even
// column count (m even); the launcher checks.
template <typename T>
__device__ __forceinline__ void lds_dma16(const void* g, C2<T>* lds_wave_base) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)lds_wave_base, 16, 0, 0);
}
template <typename T, int MODE>
__device__ __forceinline__ void cols_fill(const FFTArgs<T>& a, const ColTile<T>& t, C2<T>* s, int tid, int nthr) {
    const bool zp = MODE == 2;
    const int lg = zp ? a.lg_tx_z : a.lg_tx_y, tx = 1 << lg;
    const int nrow = zp ? a.g.nz : a.g.ny;
    const size_t rs = zp ? (size_t)a.g.ny * a.sx : (size_t)a.sx;
    const int tot = nrow << lg;
    if (t.nyq) {
        for (int e = tid; e < tot; e += nthr) {
            const int row = e >> lg, c = e & (tx - 1);
            s[e] = c < t.ncol ? t.base[row * rs + c * t.cs] : C2<T>{T(0), T(0)};
        }
        return;
    }
    constexpr int PER = 16 / (int)sizeof(C2<T>);     // complex values per lane and load (1 FP64, 2 FP32)
    const int wbase = tid & ~63;
    for (int e0 = wbase * PER; e0 < tot; e0 += nthr * PER) {
        const int e = e0 + (tid - wbase) * PER;
        const int row = e >> lg;
        int c = e & (tx - 1);
        if (c >= t.ncol) c = t.ncol - PER;            // a valid row segment; the column is never stored
        const C2<T>* src = t.base + (size_t)row * rs + c;
        if (e < tot) lds_dma16<T>(src, s + e0);
    }
}
constexpr unsigned WAIT_VMCNT0 = 0x0F70;   // s_waitcnt vmcnt(0), expcnt and lgkmcnt left alone

template <typename T, int MODE, int N>
__device__ __forceinline__ void fft_cols_pipe_loop(const FFTArgs<T>& a, int ntiles, C2<T>* s0, const C2<T>* wl,
                                                   const double* s2l, int tid, int nthr) {
    const bool zp = MODE == 2;
    const int lg = zp ? a.lg_tx_z : a.lg_tx_y, tx = 1 << lg;
    const size_t rs = zp ? (size_t)a.g.ny * a.sx : (size_t)a.sx;
    const int tot = N << lg;
    int b = (int)blockIdx.x;
    if (b < ntiles) cols_fill<T, MODE>(a, col_tile<T, MODE>(a, b), s0, tid, nthr);
    for (int i = 0; b < ntiles; ++i, b += (int)gridDim.x) {
        __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);
        __syncthreads();
        C2<T>* s = s0 + (i & 1) * tot;
        const int bn = b + (int)gridDim.x;
        if (bn < ntiles) cols_fill<T, MODE>(a, col_tile<T, MODE>(a, bn), s0 + ((i + 1) & 1) * tot, tid, nthr);
        const ColTile<T> t = col_tile<T, MODE>(a, b);
        // (no global loads from here to the stores: the symbol tables are in
        // LDS, so nothing waits for the next tile's loads).  The transforms
        // are those of cols_direct, the last radix pass storing to the
        // spectrum; the next iteration's barrier precedes the refill of this
        // buffer.
        C2<T>* const base = t.base;
        const size_t cs = t.cs;
        const int ncol = t.ncol;
        auto store = [=](int c, int row, const C2<T>& v) {
            if (c < ncol) base[row * rs + c * cs] = v;
        };
        if constexpr (MODE == 2) {
            const double* sx2l = s2l;
            const double* sy2l = s2l + a.m + 1;
            const double* sz2l = sy2l + a.g.ny;
            const double inv_ntot = a.inv_ntot;
            const int m = a.m, kx0 = t.kx0, plane0 = t.plane0;
            const bool nyq = t.nyq;
            auto divide = [=](int c, int kz, C2<T> v) -> C2<T> {
                if (c < ncol) {
                    const int kx = nyq ? m : kx0 + c;
                    const int ky = nyq ? plane0 + c : plane0;
                    const double lam = (sz2l[kz] + sy2l[ky]) + sx2l[kx];   // -lambda
                    const T f = lam == 0.0 ? T(0) : T(-inv_ntot * recip(lam));
                    v = cscale(v, f);
                }
                return v;
            };
            fft_chain_last<T, false, N, 0, false, true>(s, wl, tx, 1, lg, tid, nthr, divide);
            fft_chain_last<T, true, N, 0, true, true>(s, wl, tx, 1, lg, tid, nthr, store);
        } else {
            fft_chain_last<T, MODE == 1, N, 0, true, true>(s, wl, tx, 1, lg, tid, nthr, store);
        }
    }
}

template <typename T, int MODE>
__device__ __forceinline__ void fft_cols_pipe_body(const FFTArgs<T>& a, int ntiles) {
    extern __shared__ unsigned char smem_raw[];
    C2<T>* s0 = reinterpret_cast<C2<T>*>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const bool zp = MODE == 2;
    const int lg = zp ? a.lg_tx_z : a.lg_tx_y;
    const int nrow = zp ? a.g.nz : a.g.ny;
    C2<T>* wl = s0 + 2 * (nrow << lg);
    {
        const C2<T>* W = zp ? a.wz : a.wy;
        for (int j = tid; j < nrow; j += nthr) wl[j] = W[j];
    }
    // z pass: the three symbol tables (x: m + 1, y: ny, z: nz values) in LDS too
    double* s2l = reinterpret_cast<double*>(wl + nrow);
    if (MODE == 2) {
        const int nt = a.m + 1 + a.g.ny + a.g.nz;
        for (int j = tid; j < nt; j += nthr) s2l[j] = a.sx2[j];     // the three tables are contiguous
    }
    // one loop per transform length (the launcher only picks these lengths)
    switch (nrow) {
        case 64: fft_cols_pipe_loop<T, MODE, 64>(a, ntiles, s0, wl, s2l, tid, nthr); break;
        case 96: fft_cols_pipe_loop<T, MODE, 96>(a, ntiles, s0, wl, s2l, tid, nthr); break;
        case 128: fft_cols_pipe_loop<T, MODE, 128>(a, ntiles, s0, wl, s2l, tid, nthr); break;
        case 192: fft_cols_pipe_loop<T, MODE, 192>(a, ntiles, s0, wl, s2l, tid, nthr); break;
        case 256: fft_cols_pipe_loop<T, MODE, 256>(a, ntiles, s0, wl, s2l, tid, nthr); break;
        case 384: fft_cols_pipe_loop<T, MODE, 384>(a, ntiles, s0, wl, s2l, tid, nthr); break;
        case 512: fft_cols_pipe_loop<T, MODE, 512>(a, ntiles, s0, wl, s2l, tid, nthr); break;
        case 768: fft_cols_pipe_loop<T, MODE, 768>(a, ntiles, s0, wl, s2l, tid, nthr); break;
        case 1024: fft_cols_pipe_loop<T, MODE, 1024>(a, ntiles, s0, wl, s2l, tid, nthr); break;
        default: break;
    }
}
__host__ __device__ constexpr bool pipe_length(int n) {
    return n == 64 || n == 96 || n == 128 || n == 192 || n == 256 || n == 384 || n == 512 || n == 768 || n == 1024;
}

template <typename T, int Q, bool INV>
__device__ __forceinline__ void yz_y_phase(const FFTArgs<T>& a, C2<T> (&v)[Q], C2<T>* d, const C2<T>* wyl, int yt,
                                           int zt, int zs, int tid, int nthr) {
    const int nz = a.g.nz;
    for (int z0 = 0; z0 < nz;) {
        const int lg = min(a.lg_ca, 31 - __clz(nz - z0));
        const int nl = 1 << lg, es = nl + 1;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const unsigned zl = (unsigned)(zt + q * zs - z0);
            if (zl < (unsigned)nl) d[yt * es + zl] = v[q];
        }
        __syncthreads();
        fft_lds_inl<T, INV>(d, a.py, wyl, es, 1, lg, tid, nthr);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const unsigned zl = (unsigned)(zt + q * zs - z0);
            if (zl < (unsigned)nl) v[q] = d[yt * es + zl];
        }
        __syncthreads();
        z0 += nl;
    }
}

template <typename T, int Q>
__device__ __forceinline__ void fft_yz_body(const FFTArgs<T>& a, unsigned blk) {
    extern __shared__ unsigned char smem_raw[];
    C2<T>* s = reinterpret_cast<C2<T>*>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int ny = a.g.ny, nz = a.g.nz;
    const int kx = (int)blk;
    C2<T>* __restrict__ plane = a.spec + (size_t)kx * a.ps;
    const int yt = tid % ny, zt = tid / ny, zs = nthr / ny;
    C2<T>* wyl = s;
    C2<T>* wzl = s + ny;
    C2<T>* d = wzl + nz;
    for (int j = tid; j < ny; j += nthr) wyl[j] = a.wy[j];
    for (int j = tid; j < nz; j += nthr) wzl[j] = a.wz[j];
    C2<T> v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int z = zt + q * zs;
        v[q] = z < nz ? plane[yt + ny * z] : C2<T>{T(0), T(0)};
    }
    // (the twiddle tables are visible after the first barrier of the y phase)
    yz_y_phase<T, Q, false>(a, v, d, wyl, yt, zt, zs, tid, nthr);
    for (int y0 = 0; y0 < ny;) {
        const int lg = min(a.lg_cb, 31 - __clz(ny - y0));
        const int nl = 1 << lg, es = nl + 1;
        const unsigned yl = (unsigned)(yt - y0);
        if (yl < (unsigned)nl) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int z = zt + q * zs;
                if (z < nz) d[z * es + yl] = v[q];
            }
        }
        __syncthreads();
        fft_lds_inl<T, false>(d, a.pz, wzl, es, 1, lg, tid, nthr);
        for (int e = tid; e < (nz << lg); e += nthr) {
            const int kz = e >> lg, c = e & (nl - 1);
            const double lam = (a.sz2[kz] + a.sy2[y0 + c]) + a.sx2[kx];   // -lambda
            const T f = lam == 0.0 ? T(0) : T(-a.inv_ntot * recip(lam));
            d[kz * es + c] = cscale(d[kz * es + c], f);
        }
        __syncthreads();
        fft_lds_inl<T, true>(d, a.pz, wzl, es, 1, lg, tid, nthr);
        if (yl < (unsigned)nl) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int z = zt + q * zs;
                if (z < nz) v[q] = d[z * es + yl];
            }
        }
        __syncthreads();
        y0 += nl;
    }
    yz_y_phase<T, Q, true>(a, v, d, wyl, yt, zt, zs, tid, nthr);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int z = zt + q * zs;
        if (z < nz) plane[yt + ny * z] = v[q];
    }
}

// Plain and batched launch wrappers (see stencil.hip).
#define DNSLAB_BATCH_BLOCK(st, ns)         \
    const int s_ = batch_slot(st, ns);     \
    const unsigned blk_ = blockIdx.x - st[s_];

template <typename T>
__global__ __launch_bounds__(256) void k_ib_rhs(const IbArgs<T> a) { ib_rhs_body<T>(a, blockIdx.x); }
template <typename T>
__global__ __launch_bounds__(256) void k_ib_rhs_b(const BRec<IbArgs<T>>* __restrict__ tab,
                                                  const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_BLOCK(st, ns)
    const IbArgs<T> a = tab[s_].a;
    ib_rhs_body<T>(a, blk_);
}
template <typename T>
__global__ __launch_bounds__(1024) void k_fft_x_fwd(const FxfArgs<T> a) { fft_x_fwd_body<T>(a, blockIdx.x); }
template <typename T>
__global__ __launch_bounds__(1024) void k_fft_x_fwd_b(const BRec<FxfArgs<T>>* __restrict__ tab,
                                                      const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_BLOCK(st, ns)
    const FxfArgs<T>& a = tab[s_].a;
    fft_x_fwd_body<T>(a, blk_);
}
template <typename T>
__global__ __launch_bounds__(1024) void k_fft_x_inv(const FxiArgs<T> a) { fft_x_inv_body<T>(a, blockIdx.x); }
template <typename T>
__global__ __launch_bounds__(1024) void k_fft_x_inv_b(const BRec<FxiArgs<T>>* __restrict__ tab,
                                                      const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_BLOCK(st, ns)
    const FxiArgs<T>& a = tab[s_].a;
    fft_x_inv_body<T>(a, blk_);
}
// XCD-aware tile order for the column passes: workgroups are dealt to the 8
// XCDs round-robin by hardware id, so consecutive ids (neighbouring kx tiles
// of one plane, which share the 128-byte lines their row segments fall in)
// would land in different L2s and each fetch the whole line.  The hardware id
// is remapped so that each XCD owns a contiguous range of tiles.
__device__ __forceinline__ unsigned xcd_tile(unsigned hw, unsigned nb) {
    return DNSLAB_COL_XCD ? xcd_block(hw, nb) : hw;
}
template <typename T, int MODE, int DIRECT>
__global__ __launch_bounds__(1024) void k_fft_cols(const FFTArgs<T> a) {
    fft_cols_body<T, MODE, DIRECT>(a, xcd_tile(blockIdx.x, gridDim.x));
}
template <typename T, int MODE>
__global__ __launch_bounds__(1024) void k_fft_cols_b(const BRec<FFTArgs<T>>* __restrict__ tab,
                                                     const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_BLOCK(st, ns)
    const FFTArgs<T>& a = tab[s_].a;   // read in place: a private copy of the plan would sit in scratch
    fft_cols_body<T, MODE, 2>(a, blk_);
}

template <typename T, int MODE>
__global__ __launch_bounds__(512) void k_fft_cols_pipe(const FFTArgs<T> a, int ntiles) {
    fft_cols_pipe_body<T, MODE>(a, ntiles);
}

template <typename T, int Q>
__global__ __launch_bounds__(sizeof(T) == 8 ? YZ_THREADS : YZ_THREADS32) void k_fft_yz(const FFTArgs<T> a) {
    fft_yz_body<T, Q>(a, blockIdx.x);
}
template <typename T, int Q>
__global__ __launch_bounds__(sizeof(T) == 8 ? YZ_THREADS : YZ_THREADS32) void k_fft_yz_b(const BRec<FFTArgs<T>>* __restrict__ tab,
                                                   const unsigned* __restrict__ st, int ns) {
    DNSLAB_BATCH_BLOCK(st, ns)
    const FFTArgs<T>& a = tab[s_].a;   // read in place: a private copy of the plan would sit in scratch
    fft_yz_body<T, Q>(a, blk_);
}

// Twiddle and symbol tables of one grid, computed on the device: entry i of
// the twiddle block is W_n^j = e^{-2 pi i j / n} for (n, j) = (m, j < m),
// (ny, j < ny), (nz, j < nz), (nx, j <= m) in turn; entry k of the symbol
// block is sin^2(2 pi j / N) / dx^2 for (N, j) = (nx, j <= m), (ny, j < ny),
// (nz, j < nz), exactly zero where 2j is a multiple of N (the null set of
// Section 2.2's central-difference symbol).  One thread per entry.
template <typename T>
__global__ __launch_bounds__(256) void k_fft_tables(C2<T>* __restrict__ w, double* __restrict__ s2, int nx, int ny,
                                                    int nz, double dx, double dy, double dz) {
    const int m = nx / 2;
    const int nw = 2 * m + 1 + ny + nz, nsym = m + 1 + ny + nz;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nw) {
        int n, j;
        if (i < m) { n = m; j = i; }
        else if (i < m + ny) { n = ny; j = i - m; }
        else if (i < m + ny + nz) { n = nz; j = i - m - ny; }
        else { n = nx; j = i - m - ny - nz; }
        double sn, cs;
        sincospi(2.0 * (double)j / (double)n, &sn, &cs);
        w[i] = C2<T>{(T)cs, (T)(-sn)};
    } else if (i < nw + nsym) {
        const int k = i - nw;
        int n, j;
        double h;
        if (k < m + 1) { n = nx; j = k; h = dx; }
        else if (k < m + 1 + ny) { n = ny; j = k - m - 1; h = dy; }
        else { n = nz; j = k - m - 1 - ny; h = dz; }
        double v = 0.0;
        if ((2LL * j) % n != 0) {
            const double sn = sinpi(2.0 * (double)j / (double)n);
            v = sn * sn / (h * h);
        }
        s2[k] = v;
    }
}

inline int round64(int t) { return ((t + 63) / 64) * 64; }

}  // namespace

AxisPlan make_axis_plan(int n) {
    AxisPlan p = {};
    p.n = n;
    int a = 0, b = 0, m = n;
    while (m > 1 && m % 2 == 0) { m /= 2; ++a; }
    while (m > 1 && m % 3 == 0) { m /= 3; ++b; }
    if (m != 1 || n < 1) { p.npass = -1; return p; }
    int np = 0;
    int eights = a / 3, rest = a % 3;
    if (rest == 1 && eights >= 1) {           // 2^(3e+1) = 8^(e-1) * 4 * 4
        for (int i = 0; i < eights - 1; ++i) p.rad[np++] = 8;
        p.rad[np++] = 4;
        p.rad[np++] = 4;
    } else {
        for (int i = 0; i < eights; ++i) p.rad[np++] = 8;
        if (rest == 2) p.rad[np++] = 4;
        if (rest == 1) p.rad[np++] = 2;
    }
    for (int i = 0; i < b; ++i) p.rad[np++] = 3;
    p.npass = np;
    p.tpl = np > 0 ? n / p.rad[0] : 1;
    return p;
}

template <typename T>
hipError_t launch_ib_rhs(const IBList& ib, const Grid& g, const T* p, T* r, T* r0s, int first, hipStream_t s,
                         Recorder* rec) {
    if (ib.n <= 0) return hipSuccess;
    IbArgs<T> a;
    a.ib = ib;
    a.g = g;
    a.p = p;
    a.r = r;
    a.r0s = r0s;
    a.first = first;
    const dim3 grid((ib.n + 256 * IB_CPT - 1) / (256 * IB_CPT)), block(256);
    if (rec) {
        record_launch(rec, kind_code(KK_IB, 0, sizeof(T) == 4), grid, block, 0, a);
        return hipSuccess;
    }
    hipLaunchKernelGGL((k_ib_rhs<T>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_x_fwd(const FFTArgs<T>& a, const T* r, hipStream_t s, Recorder* rec) {
    const int nl = 1 << a.nl_x;
    const int nlines = a.g.ny * a.g.nz;
    dim3 grid((nlines + nl - 1) / nl);
    dim3 block(round64(std::min(1024, nl * a.px.tpl * DNSLAB_FFT_TPL_MUL)));
    size_t lds = ((size_t)nl * a.ls_x + (a.xtw_lds ? 2 * a.m + 1 : 0)) * sizeof(C2<T>);
    FxfArgs<T> b;
    b.f = a;
    b.r = r;
    if (rec) {
        record_launch(rec, kind_code(KK_FXF, 0, sizeof(T) == 4), grid, block, lds, b);
        return hipSuccess;
    }
    hipLaunchKernelGGL((k_fft_x_fwd<T>), grid, block, lds, s, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_x_inv(const FFTArgs<T>& a, T* p, hipStream_t s, Recorder* rec) {
    const int nl = 1 << a.nl_x;
    const int nlines = a.g.ny * a.g.nz;
    dim3 grid((nlines + nl - 1) / nl);
    dim3 block(round64(std::min(1024, nl * a.px.tpl * DNSLAB_FFT_TPL_MUL)));
    size_t lds = ((size_t)nl * a.ls_x + (a.xtw_lds ? 2 * a.m + 1 : 0)) * sizeof(C2<T>);
    FxiArgs<T> b;
    b.f = a;
    b.p = p;
    if (rec) {
        record_launch(rec, kind_code(KK_FXI, 0, sizeof(T) == 4), grid, block, lds, b);
        return hipSuccess;
    }
    hipLaunchKernelGGL((k_fft_x_inv<T>), grid, block, lds, s, b);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_cols(const FFTArgs<T>& a, int mode, hipStream_t s, Recorder* rec) {
    const bool zp = mode == 2;
    const int lg = zp ? a.lg_tx_z : a.lg_tx_y, tx = 1 << lg;
    const int nrow = zp ? a.g.nz : a.g.ny, nplane = zp ? a.g.ny : a.g.nz;
    const int ntile = (a.m + tx - 1) / tx;
    const int nblocks = ntile * nplane + (nplane + tx - 1) / tx;
    const AxisPlan& ap = zp ? a.pz : a.py;
    dim3 block(round64(std::min(1024, tx * ap.tpl * DNSLAB_FFT_TPL_MUL)));
    // every first-pass butterfly needs a thread (longer lines than the block
    // can cover are refused rather than transformed in part)
    if ((long long)block.x < (long long)tx * ap.tpl) return hipErrorInvalidValue;
    size_t lds = ((size_t)tx * nrow + nrow) * sizeof(C2<T>);
    // the pipelined pass (plain launches): two tile buffers, each block
    // walking at least two tiles
    const size_t lds_pipe = ((size_t)2 * tx * nrow + nrow) * sizeof(C2<T>) +
                            (mode == 2 ? (size_t)(a.m + 1 + a.g.ny + a.g.nz) * sizeof(double) : 0);
    const int per = 16 / (int)sizeof(C2<T>);
    const bool fits = a.ps == 0 && tx >= per && (sizeof(T) == 8 || a.m % 2 == 0) && lds_pipe <= 160 * 1024 &&
                      (size_t)nrow * tx >= (size_t)block.x * per && block.x <= 512 && pipe_length(nrow);
    if (!rec && fits && a.col_pipe != 0) {
        const int bpc = (int)std::max<size_t>(1, (160 * 1024) / lds_pipe);
        const int grid = std::min(nblocks, 256 * bpc);
        if (a.col_pipe == 1 || nblocks >= 2 * grid) {
            if (mode == 0) hipLaunchKernelGGL((k_fft_cols_pipe<T, 0>), dim3(grid), block, lds_pipe, s, a, nblocks);
            else if (mode == 1) hipLaunchKernelGGL((k_fft_cols_pipe<T, 1>), dim3(grid), block, lds_pipe, s, a, nblocks);
            else hipLaunchKernelGGL((k_fft_cols_pipe<T, 2>), dim3(grid), block, lds_pipe, s, a, nblocks);
            return hipGetLastError();
        }
    }
    if (rec) {
        record_launch(rec, kind_code(KK_COLS, mode, sizeof(T) == 4), dim3(nblocks), block, lds, a);
        return hipSuccess;
    }
    const bool direct = DNSLAB_COL_DIRECT && pipe_length(nrow);
    if (direct) {
        if (mode == 0) hipLaunchKernelGGL((k_fft_cols<T, 0, 1>), dim3(nblocks), block, lds, s, a);
        else if (mode == 1) hipLaunchKernelGGL((k_fft_cols<T, 1, 1>), dim3(nblocks), block, lds, s, a);
        else hipLaunchKernelGGL((k_fft_cols<T, 2, 1>), dim3(nblocks), block, lds, s, a);
    } else {
        if (mode == 0) hipLaunchKernelGGL((k_fft_cols<T, 0, 0>), dim3(nblocks), block, lds, s, a);
        else if (mode == 1) hipLaunchKernelGGL((k_fft_cols<T, 1, 0>), dim3(nblocks), block, lds, s, a);
        else hipLaunchKernelGGL((k_fft_cols<T, 2, 0>), dim3(nblocks), block, lds, s, a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_y(const FFTArgs<T>& a, bool inverse, hipStream_t s, Recorder* rec) {
    return launch_cols<T>(a, inverse ? 1 : 0, s, rec);
}

template <typename T>
hipError_t launch_fft_z_solve(const FFTArgs<T>& a, hipStream_t s, Recorder* rec) {
    return launch_cols<T>(a, 2, s, rec);
}

template <typename T>
hipError_t launch_fft_yz_solve(const FFTArgs<T>& a, hipStream_t s, Recorder* rec) {
    const int nthr = yz_threads(a.g.ny, sizeof(T) == 4);
    const int qi = nthr > 0 ? yz_instance(sizeof(T) == 4, nthr, (long long)a.g.ny * a.g.nz) : -1;
    if (a.ps != a.g.ny * a.g.nz || nthr <= 0 || qi < 0 ||
        ((long long)a.py.tpl << a.lg_ca) > nthr || ((long long)a.pz.tpl << a.lg_cb) > nthr)
        return hipErrorInvalidValue;
    const dim3 grid(a.m + 1), block(nthr);
    const size_t lds = ((size_t)a.g.ny + a.g.nz +
                        std::max((size_t)a.g.ny * ((1 << a.lg_ca) + 1), (size_t)a.g.nz * ((1 << a.lg_cb) + 1))) *
                       sizeof(C2<T>);
    // kind modes 3 + i: the instance with yz_q<T>(i) values per thread
    if (rec) {
        record_launch(rec, kind_code(KK_COLS, 3 + qi, sizeof(T) == 4), grid, block, lds, a);
        return hipSuccess;
    }
    switch (qi) {
        case 0: hipLaunchKernelGGL((k_fft_yz<T, yz_q<T>(0)>), grid, block, lds, s, a); break;
        case 1: hipLaunchKernelGGL((k_fft_yz<T, yz_q<T>(1)>), grid, block, lds, s, a); break;
        case 2: hipLaunchKernelGGL((k_fft_yz<T, yz_q<T>(2)>), grid, block, lds, s, a); break;
        case 3: hipLaunchKernelGGL((k_fft_yz<T, yz_q<T>(3)>), grid, block, lds, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_tables(C2<T>* w, double* s2, const Grid& g, hipStream_t s) {
    const int m = g.nx / 2;
    const int total = (2 * m + 1 + g.ny + g.nz) + (m + 1 + g.ny + g.nz);
    hipLaunchKernelGGL((k_fft_tables<T>), dim3((total + 255) / 256), dim3(256), 0, s, w, s2, g.nx, g.ny, g.nz,
                       g.d[0], g.d[1], g.d[2]);
    return hipGetLastError();
}

namespace {
template <typename T>
hipError_t fft_batched_typed(int base, int mode, const void* tab, const unsigned* st, int ns, unsigned nb, dim3 blk,
                             size_t lds, hipStream_t s) {
    const dim3 grid(nb);
    switch (base) {
        case KK_IB:
            hipLaunchKernelGGL((k_ib_rhs_b<T>), grid, blk, 0, s, (const BRec<IbArgs<T>>*)tab, st, ns);
            break;
        case KK_FXF:
            hipLaunchKernelGGL((k_fft_x_fwd_b<T>), grid, blk, lds, s, (const BRec<FxfArgs<T>>*)tab, st, ns);
            break;
        case KK_FXI:
            hipLaunchKernelGGL((k_fft_x_inv_b<T>), grid, blk, lds, s, (const BRec<FxiArgs<T>>*)tab, st, ns);
            break;
        case KK_COLS: {
            auto t = (const BRec<FFTArgs<T>>*)tab;
            if (mode == 0) hipLaunchKernelGGL((k_fft_cols_b<T, 0>), grid, blk, lds, s, t, st, ns);
            else if (mode == 1) hipLaunchKernelGGL((k_fft_cols_b<T, 1>), grid, blk, lds, s, t, st, ns);
            else if (mode == 2) hipLaunchKernelGGL((k_fft_cols_b<T, 2>), grid, blk, lds, s, t, st, ns);
            else if (mode == 3) hipLaunchKernelGGL((k_fft_yz_b<T, yz_q<T>(0)>), grid, blk, lds, s, t, st, ns);
            else if (mode == 4) hipLaunchKernelGGL((k_fft_yz_b<T, yz_q<T>(1)>), grid, blk, lds, s, t, st, ns);
            else if (mode == 5) hipLaunchKernelGGL((k_fft_yz_b<T, yz_q<T>(2)>), grid, blk, lds, s, t, st, ns);
            else if (mode == 6) hipLaunchKernelGGL((k_fft_yz_b<T, yz_q<T>(3)>), grid, blk, lds, s, t, st, ns);
            else return hipErrorInvalidValue;
            break;
        }
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_batched_fft(int kind, const void* tab, const unsigned* st, int ns, unsigned nb, dim3 blk,
                              size_t lds, hipStream_t s) {
    const int base = kind >> 8, mode = (kind >> 1) & 127, fp32 = kind & 1;
    return fp32 ? fft_batched_typed<float>(base, mode, tab, st, ns, nb, blk, lds, s)
                : fft_batched_typed<double>(base, mode, tab, st, ns, nb, blk, lds, s);
}

#define DNSLAB_INST(T)                                                                                  \
    template hipError_t launch_fft_x_fwd<T>(const FFTArgs<T>&, const T*, hipStream_t, Recorder*);       \
    template hipError_t launch_ib_rhs<T>(const IBList&, const Grid&, const T*, T*, T*, int, hipStream_t,  \
                                         Recorder*);                                                    \
    template hipError_t launch_fft_x_inv<T>(const FFTArgs<T>&, T*, hipStream_t, Recorder*);              \
    template hipError_t launch_fft_y<T>(const FFTArgs<T>&, bool, hipStream_t, Recorder*);                \
    template hipError_t launch_fft_z_solve<T>(const FFTArgs<T>&, hipStream_t, Recorder*);                \
    template hipError_t launch_fft_yz_solve<T>(const FFTArgs<T>&, hipStream_t, Recorder*);               \
    template hipError_t launch_fft_tables<T>(C2<T>*, double*, const Grid&, hipStream_t);
DNSLAB_INST(double)
DNSLAB_INST(float)
#undef DNSLAB_INST

}  // namespace dnslab
