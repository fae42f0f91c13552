// Launch interface of the stencil kernels (stencil.hip).
#pragma once
#include "common.h"

namespace dnslab {

// Stage modes of the classical RK4 (Section 2.1), with acc the running sum
// u^n + dt/6 k1 + dt/3 k2 + dt/3 k3.
enum StageMode {
    ST_FIRST = 0,   // k1 = F(u^n); acc = u^n + dt/6 k1; out = u^n + dt/2 k1
    ST_HALF = 1,    // k2 = F(u1);  acc += dt/3 k2;      out = u^n + dt/2 k2
    ST_FULL = 2,    // k3 = F(u2);  acc += dt/3 k3;      out = u^n + dt k3
    ST_LAST = 3,    // k4 = F(u3);  out = acc + dt/6 k4 (scalar: times beta)
    ST_RHS = 4,     // out = F(in)
};

template <typename T>
struct MomArgs {
    const T* us[3];   // stage input (read with neighbours)
    const T* un[3];   // u^n (ST_HALF, ST_FULL)
    T* acc[3];
    T* out[3];
    const uint8_t* flags;
    const double* dtp;   // device dt (NULL: use dt)
    double dt;
    Forcing frc;
    double nu;
    double body[3];
    Grid g;
    int kc;              // cells per thread along z
};

// Two RK4 stages in one pass (the stages need no pressure: the projection
// comes once per step).  Pair 0: k1 = F(u^n), u1 = u^n + dt/2 k1 on the tile
// and a one-cell ring around it, k2 = F(u1) on the tile; writes
// acc = (u^n + dt/6 k1) + dt/3 k2 and u2 = u^n + dt/2 k2.  Pair 1: k3 = F(u2),
// u3 = u^n + dt k3 on tile and ring, k4 = F(u3); writes
// u* = (acc + dt/3 k3) + dt/6 k4.  Each value is computed with the same
// expressions as by the single-stage kernels.
template <typename T>
struct MomPairArgs {
    const T* vin[3];    // stage input: u^n (pair 0), u2 (pair 1), read with a radius-2 halo
    const T* un[3];     // u^n (pair 1: on the tile and its ring)
    const T* accin[3];  // acc after stage 2 (pair 1)
    T* acc[3];          // pair 0: acc after stage 2
    T* out[3];          // pair 0: u2; pair 1: u*
    const uint8_t* flags;
    const double* dtp;
    double dt;
    Forcing frc;
    double nu;
    double body[3];
    Grid g;
    int kc;
};

template <typename T>
struct ScaArgs {
    const T* cs;      // stage input (read with neighbours)
    const T* cn;      // c^n (ST_HALF, ST_FULL)
    T* acc;
    T* out;
    const T* u[3];    // frozen velocity
    const uint8_t* flags;
    const double* dtp;
    double dt;
    Forcing frc;
    double alpha;
    Grid g;
    int kc;
    PartSoA part;     // ST_FIRST: div^2 partials; ST_LAST: CO2 diagnostics partials (p NULL: none)
};

// Two scalar RK4 stages in one pass, as MomPairArgs for the momentum: pair 0
// k1 = G(c^n) on tile and ring, c1 = c^n + dt/2 k1, k2 = G(c1); writes
// acc = (c^n + dt/6 k1) + dt/3 k2 and c2 = c^n + dt/2 k2 (partials: div u
// squared).  Pair 1: k3 = G(c2), c3 = c^n + dt k3 on tile and ring, k4 = G(c3);
// writes c* = beta ((acc + dt/3 k3) + dt/6 k4) (partials: CO2 mass and room
// sums).  The velocity is frozen.
template <typename T>
struct ScaPairArgs {
    const T* cin;     // stage input: c^n (pair 0), c2 (pair 1), read with a radius-2 halo
    const T* cn;      // c^n (pair 1: tile and ring)
    const T* accin;   // acc after stage 2 (pair 1)
    T* acc;           // pair 0: acc after stage 2
    T* out;           // pair 0: c2; pair 1: c*
    const T* u[3];
    const uint8_t* flags;
    const double* dtp;
    double dt;
    Forcing frc;
    double alpha;
    Grid g;
    int kc;
    PartSoA part;
};

template <typename T>
struct FiltArgs {
    const T* in[3];
    T* out[3];
    int nf;           // 3: the velocity (partials: kinetic energy, Courant rate); 1: a scalar (CO2 partials)
    const uint8_t* flags;
    Grid g;
    int kc;
    PartSoA part;     // diagnostics partials of the outputs (p NULL: none)
};

template <typename T>
struct CorrArgs {
    const T* us[3];   // u* (pointwise; may alias out)
    T* out[3];
    const T* p;
    const uint8_t* flags;
    Grid g;
    int kc;
    PartSoA part;     // kinetic energy and Courant rate partials of out (p NULL: none)
};

template <typename T>
struct DivArgs {
    const T* u[3];
    T* out;
    Grid g;
    int kc;
};

// FP64 refinement of the last pressure solve of the FP32 form.
// res = div u* + div((1-beta) grad p3) - Lap_h p4, evaluated in FP64 from the
// FP32 fields (Lap_h = div grad with central differences), stored as FP32.
struct RefineResArgs {
    const float* us[3];
    const float* p3;       // pressure iterate entering the last solve
    const float* p4;       // result of the last FP32 solve
    const uint8_t* flags;
    float* res;
    Grid g;
    int kc;
    IBList ib;             // the cells next to a solid (their residual has the IB term)
};
// u = beta (u* - grad(p4 + dp)) and p = p4 + dp, in FP64 arithmetic.
struct RefineCorrArgs {
    const float* us[3];    // may alias out
    float* out[3];
    const float* p4;
    const float* dp;
    float* p;
    const uint8_t* flags;
    Grid g;
    int kc;
    PartSoA part;          // as CorrArgs::part
};
hipError_t launch_refine_res(const RefineResArgs& a, const struct StencilLaunch& L, hipStream_t s,
                             Recorder* rec = nullptr);
hipError_t launch_refine_correct(const RefineCorrArgs& a, const struct StencilLaunch& L, hipStream_t s,
                                 Recorder* rec = nullptr);

// Launch geometry shared by all z-marching stencil kernels.
struct StencilLaunch {
    dim3 grid, block;
    int kc;
    int nblocks;
};
// rows: block height for a 64-wide block (the block has 64 * rows threads);
// cells_x: cells per thread along x (1, or 2 for the pair kernels).
StencilLaunch stencil_launch(const Grid& g, int rows, int kc, int cells_x);

// Every launch_* issues one kernel on stream s, or, when rec is non-NULL,
// records the launch (for batched replay by the pool) without issuing it.
template <typename T> hipError_t launch_mom_stage(int mode, const MomArgs<T>& a, const StencilLaunch& L, hipStream_t s,
                                                  Recorder* rec = nullptr);
// Block height of the radius-3 filter and of the velocity correction
// (64 x DNSLAB_FROWS tiles; their register-ring forms are compiled for this
// height).  16 rows cut the filter's x/y halo from 0.91 to 0.5 of the tile:
// on 1024x512x256 the FP64 filter went from 1792 to 1637 us and the
// correction from 1619 to 1532 us against 64 x 8.
#ifndef DNSLAB_FROWS
#define DNSLAB_FROWS 16
#endif
// Rows of the 64-wide tile of the stage-pair kernels (a compile-time tile
// shape: the kernels' LDS offsets are immediates).
#ifndef DNSLAB_PROWS
#define DNSLAB_PROWS 8
#endif
// The pair kernels need the 64 x DNSLAB_PROWS tile to divide the grid in x
// and y (mom_pair_supported); otherwise the single-stage kernels run.
bool mom_pair_supported(const Grid& g, const StencilLaunch& L);
template <typename T> hipError_t launch_mom_pair(int pair, const MomPairArgs<T>& a, const StencilLaunch& L,
                                                 hipStream_t s, Recorder* rec = nullptr);
template <typename T> hipError_t launch_sca_pair(int pair, const ScaPairArgs<T>& a, const StencilLaunch& L,
                                                 hipStream_t s, Recorder* rec = nullptr);
template <typename T> hipError_t launch_sca_stage(int mode, const ScaArgs<T>& a, const StencilLaunch& L, hipStream_t s,
                                                  Recorder* rec = nullptr);
template <typename T> hipError_t launch_filter(const FiltArgs<T>& a, const StencilLaunch& L, hipStream_t s,
                                               Recorder* rec = nullptr);
template <typename T> hipError_t launch_correct(const CorrArgs<T>& a, const StencilLaunch& L, hipStream_t s,
                                                Recorder* rec = nullptr);
template <typename T> hipError_t launch_div(const DivArgs<T>& a, const StencilLaunch& L, hipStream_t s,
                                            Recorder* rec = nullptr);
template <typename T> hipError_t launch_rate(const T* u, const T* v, const T* w, const Grid& g,
                                             PartSoA part, const StencilLaunch& L, hipStream_t s);

// End of a step's velocity update (one block): reduce the Courant rate
// partials of the new velocity, advance t and the step count, keep the step's
// dt and starting rate for its diagnostics record, and set the next dt.
struct AdvanceArgs {
    PartSoA part;
    int np;
    StepScalars* sc;
};
hipError_t launch_advance(const AdvanceArgs& a, hipStream_t s, Recorder* rec = nullptr);

// Diagnostics record of the step just advanced (one block): reduce the kinetic
// energy, CO2 and divergence partials and write the record into the ring.
struct DiagArgs {
    PartSoA part;
    int np_vel, np_sca, np_div;
    StepScalars* sc;
    DiagRec* ring;
    int ring_cap;
    double dv;
};
hipError_t launch_diag(const DiagArgs& a, hipStream_t s, Recorder* rec = nullptr);

// Batched replay of one recorded position over ns scenarios: tab holds ns
// BRec<Args> entries (device), starts the ns+1 block offsets (device).
hipError_t launch_batched_stencil(int kind, const void* tab, const unsigned* starts, int ns, unsigned total_blocks,
                                  dim3 block, size_t lds, hipStream_t s);
// Reduce Courant partials only: sets sc->rate and the next dt.
hipError_t launch_set_rate(PartSoA part, int np, StepScalars* sc, hipStream_t s);

}  // namespace dnslab
