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
// coalesced.
#include "fft.h"

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
__device__ __forceinline__ void stockham_pass(C2<T>* s, int n, int ns, const C2<T>* __restrict__ W, int es,
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
__device__ void fft_lds(C2<T>* s, const AxisPlan& ap, const C2<T>* __restrict__ W, int es, int ls, int lg_nl,
                        int tid, int nthr) {
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

// div((1 - beta) grad p) at cell (i, j, k) with central differences and the
// mask taken at the face neighbours (only called for flagged cells).
template <typename T>
__device__ T ib_term(const Grid& g, const T* __restrict__ p, const uint8_t* __restrict__ fl, int i, int j, int k) {
    T acc = T(0);
    const int nn[3] = {g.nx, g.ny, g.nz};
    const int c0[3] = {i, j, k};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int cc[3] = {c0[0], c0[1], c0[2]};
        auto at = [&](int off) -> unsigned {
            cc[a] = wrap(c0[a] + off, nn[a]);
            const unsigned r = (unsigned)cc[0] + (unsigned)g.nx * ((unsigned)cc[1] + (unsigned)g.ny * cc[2]);
            cc[a] = c0[a];
            return r;
        };
        const T h = T(g.inv2d[a]);
        const unsigned ip = at(1), im = at(-1);
        if (!(fl[ip] & F_FLUID)) acc += ((p[at(2)] - p[at(0)]) * h) * h;
        if (!(fl[im] & F_FLUID)) acc -= ((p[at(0)] - p[at(-2)]) * h) * h;
    }
    return acc;
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

template <typename T>
__global__ __launch_bounds__(1024) void k_fft_x_fwd(const FFTArgs<T> a, const T* __restrict__ r0,
                                                    const T* __restrict__ p, const uint8_t* __restrict__ flags) {
    extern __shared__ unsigned char smem_raw[];
    C2<T>* s = reinterpret_cast<C2<T>*>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lg = a.nl_x, m = a.m, ls = a.ls_x;
    const int line0 = blockIdx.x << lg;
    const int nlines = a.g.ny * a.g.nz;
    const int nx = a.g.nx;
    for (int e = tid; e < (m << lg); e += nthr) {
        const int l = e / m;
        const int n = e - l * m;
        const int L = line0 + l;
        C2<T> z = {T(0), T(0)};
        if (L < nlines) {
            const unsigned idx = (unsigned)L * (unsigned)nx + 2u * (unsigned)n;
            z = *reinterpret_cast<const C2<T>*>(r0 + idx);
            if (flags) {
                const uint8_t f0 = flags[idx], f1 = flags[idx + 1];
                if ((f0 | f1) & F_NEAR_SOLID) {
                    const int j = L % a.g.ny, k = L / a.g.ny;
                    if (f0 & F_NEAR_SOLID) z.x += ib_term(a.g, p, flags, 2 * n, j, k);
                    if (f1 & F_NEAR_SOLID) z.y += ib_term(a.g, p, flags, 2 * n + 1, j, k);
                }
            }
        }
        s[l * ls + n] = z;
    }
    __syncthreads();
    fft_lds<T, false>(s, a.px, a.wx, 1, ls, lg, tid, nthr);
    const int half = m / 2 + 1;
    for (int e = tid; e < (half << lg); e += nthr) {
        const int l = e / half;
        const int k = e - l * half;
        const int L = line0 + l;
        if (L >= nlines) continue;
        const C2<T>* zl = s + l * ls;
        C2<T>* out = a.spec + (size_t)L * a.sx;
        const C2<T> za = zl[k];
        const C2<T> zb = zl[k == 0 ? 0 : m - k];
        out[k] = r2c_post(za, zb, a.tw[k]);
        if (m - k != k) out[m - k] = r2c_post(zb, za, a.tw[m - k]);
    }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_fft_x_inv(const FFTArgs<T> a, T* __restrict__ p) {
    extern __shared__ unsigned char smem_raw[];
    C2<T>* s = reinterpret_cast<C2<T>*>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lg = a.nl_x, m = a.m, ls = a.ls_x;
    const int line0 = blockIdx.x << lg;
    const int nlines = a.g.ny * a.g.nz;
    const int nx = a.g.nx;
    const int m1 = m + 1;
    for (int e = tid; e < (m1 << lg); e += nthr) {
        const int l = e / m1;
        const int k = e - l * m1;
        const int L = line0 + l;
        s[l * ls + k] = L < nlines ? a.spec[(size_t)L * a.sx + k] : C2<T>{T(0), T(0)};
    }
    __syncthreads();
    const int half = m / 2 + 1;
    for (int e = tid; e < (half << lg); e += nthr) {
        const int l = e / half;
        const int k = e - l * half;
        C2<T>* zl = s + l * ls;
        C2<T> xa = zl[k], xb = zl[m - k];
        if (k == 0) { xa.y = T(0); xb.y = T(0); }   // the real transform ignores Im X[0], Im X[m]
        const C2<T> za = c2r_pre(xa, xb, a.tw[k]);
        if (k != 0 && m - k != k) zl[m - k] = c2r_pre(xb, xa, a.tw[m - k]);
        zl[k] = za;
    }
    __syncthreads();
    fft_lds<T, true>(s, a.px, a.wx, 1, ls, lg, tid, nthr);
    for (int e = tid; e < (m << lg); e += nthr) {
        const int l = e / m;
        const int n = e - l * m;
        const int L = line0 + l;
        if (L < nlines)
            *reinterpret_cast<C2<T>*>(p + (unsigned)L * (unsigned)nx + 2u * (unsigned)n) = s[l * ls + n];
    }
}

template <typename T, bool INV>
__global__ __launch_bounds__(1024) void k_fft_y(const FFTArgs<T> a) {
    extern __shared__ unsigned char smem_raw[];
    C2<T>* s = reinterpret_cast<C2<T>*>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lg = a.lg_tx_y, tx = 1 << lg;
    const int c0 = blockIdx.x << lg;
    const int kz = blockIdx.y;
    const int ny = a.g.ny, ncols = a.m + 1;
    C2<T>* base = a.spec + (size_t)kz * ny * a.sx + c0;
    const int tot = ny << lg;
    for (int e = tid; e < tot; e += nthr) {
        const int row = e >> lg, c = e & (tx - 1);
        s[e] = (c0 + c < ncols) ? base[(size_t)row * a.sx + c] : C2<T>{T(0), T(0)};
    }
    __syncthreads();
    fft_lds<T, INV>(s, a.py, a.wy, tx, 1, lg, tid, nthr);
    for (int e = tid; e < tot; e += nthr) {
        const int row = e >> lg, c = e & (tx - 1);
        if (c0 + c < ncols) base[(size_t)row * a.sx + c] = s[e];
    }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_fft_z_solve(const FFTArgs<T> a) {
    extern __shared__ unsigned char smem_raw[];
    C2<T>* s = reinterpret_cast<C2<T>*>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lg = a.lg_tx_z, tx = 1 << lg;
    const int c0 = blockIdx.x << lg;
    const int ky = blockIdx.y;
    const int ny = a.g.ny, nz = a.g.nz, ncols = a.m + 1;
    C2<T>* base = a.spec + (size_t)ky * a.sx + c0;
    const size_t rs = (size_t)ny * a.sx;
    const int tot = nz << lg;
    for (int e = tid; e < tot; e += nthr) {
        const int row = e >> lg, c = e & (tx - 1);
        s[e] = (c0 + c < ncols) ? base[row * rs + c] : C2<T>{T(0), T(0)};
    }
    __syncthreads();
    fft_lds<T, false>(s, a.pz, a.wz, tx, 1, lg, tid, nthr);
    const double syk = a.sy2[ky];
    for (int e = tid; e < tot; e += nthr) {
        const int kz = e >> lg, c = e & (tx - 1);
        const int kx = c0 + c;
        if (kx < ncols) {
            const double lam = (a.sz2[kz] + syk) + a.sx2[kx];   // -lambda
            const T f = lam == 0.0 ? T(0) : T(-a.inv_ntot / lam);
            s[e] = cscale(s[e], f);
        }
    }
    __syncthreads();
    fft_lds<T, true>(s, a.pz, a.wz, tx, 1, lg, tid, nthr);
    for (int e = tid; e < tot; e += nthr) {
        const int row = e >> lg, c = e & (tx - 1);
        if (c0 + c < ncols) base[row * rs + c] = s[e];
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
hipError_t launch_fft_x_fwd(const FFTArgs<T>& a, const T* r0, const T* p, const uint8_t* flags, hipStream_t s) {
    const int nl = 1 << a.nl_x;
    const int nlines = a.g.ny * a.g.nz;
    dim3 grid((nlines + nl - 1) / nl);
    dim3 block(round64(nl * a.px.tpl));
    size_t lds = (size_t)nl * a.ls_x * sizeof(C2<T>);
    hipLaunchKernelGGL((k_fft_x_fwd<T>), grid, block, lds, s, a, r0, p, flags);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_x_inv(const FFTArgs<T>& a, T* p, hipStream_t s) {
    const int nl = 1 << a.nl_x;
    const int nlines = a.g.ny * a.g.nz;
    dim3 grid((nlines + nl - 1) / nl);
    dim3 block(round64(nl * a.px.tpl));
    size_t lds = (size_t)nl * a.ls_x * sizeof(C2<T>);
    hipLaunchKernelGGL((k_fft_x_inv<T>), grid, block, lds, s, a, p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_y(const FFTArgs<T>& a, bool inverse, hipStream_t s) {
    const int tx = 1 << a.lg_tx_y;
    dim3 grid((a.m + 1 + tx - 1) / tx, a.g.nz);
    dim3 block(round64(tx * a.py.tpl));
    size_t lds = (size_t)tx * a.g.ny * sizeof(C2<T>);
    if (inverse) hipLaunchKernelGGL((k_fft_y<T, true>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_fft_y<T, false>), grid, block, lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_z_solve(const FFTArgs<T>& a, hipStream_t s) {
    const int tx = 1 << a.lg_tx_z;
    dim3 grid((a.m + 1 + tx - 1) / tx, a.g.ny);
    dim3 block(round64(tx * a.pz.tpl));
    size_t lds = (size_t)tx * a.g.nz * sizeof(C2<T>);
    hipLaunchKernelGGL((k_fft_z_solve<T>), grid, block, lds, s, a);
    return hipGetLastError();
}

#define DNSLAB_INST(T)                                                                                      \
    template hipError_t launch_fft_x_fwd<T>(const FFTArgs<T>&, const T*, const T*, const uint8_t*, hipStream_t); \
    template hipError_t launch_fft_x_inv<T>(const FFTArgs<T>&, T*, hipStream_t);                            \
    template hipError_t launch_fft_y<T>(const FFTArgs<T>&, bool, hipStream_t);                              \
    template hipError_t launch_fft_z_solve<T>(const FFTArgs<T>&, hipStream_t);
DNSLAB_INST(double)
DNSLAB_INST(float)
#undef DNSLAB_INST

}  // namespace dnslab
