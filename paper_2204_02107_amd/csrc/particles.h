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

}  // namespace dnslab
