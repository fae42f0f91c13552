// Launch interface of the particle kernel (particles.hip).
#pragma once
#include "common.h"

namespace dnslab {

// One implicit-Euler step of n particles (Section 2.3) in the velocity field
// (u, v, w) of grid g.  Positions and velocities are FP64, structure of arrays,
// updated in place; dt from *dtp when dtp is non-NULL.
template <typename T>
struct ParticleArgs {
    const T* u;
    const T* v;
    const T* w;
    Grid g;
    double box[3];         // periodic box lengths
    double* px;
    double* py;
    double* pz;
    double* vx;
    double* vy;
    double* vz;
    const double* diam;    // particle diameters
    long long n;
    double nu, rho_p, rho_f;
    double g_acc[3];       // gravitational acceleration
    const double* dtp;
    double dt;
};

template <typename T>
hipError_t launch_particles(const ParticleArgs<T>& a, hipStream_t s);

// Reordering of particles by the cell that holds them (so that neighbouring
// threads of the step kernel gather from neighbouring cells).  Scratch sizes
// for n particles; the buffers are the caller's.
struct ParticleSortScratch {
    unsigned* keys[2];     // n cell indices each
    unsigned* vals[2];     // n particle indices each
    double* tmp;           // n doubles
    void* sort_tmp;        // radix-sort counts and scan totals
    size_t sort_bytes;
};
// Bytes of radix-sort counts and scan totals for n particles.
hipError_t particle_sort_bytes(long long n, size_t* bytes);
// Largest n the sort handles (its scan has two levels).
long long particle_sort_max();
// Stable sort of the n particles (SoA pos, vel: 3 n doubles each; diam: n)
// by the linear index of the containing cell; every array is permuted in place.
hipError_t sort_particles(const Grid& g, long long n, double* pos, double* vel, double* diam,
                          const ParticleSortScratch& s, hipStream_t st);

}  // namespace dnslab
