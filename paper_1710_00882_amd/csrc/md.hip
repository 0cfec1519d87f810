// Kernels of the molecular-dynamics driver (velocity-Verlet NVE around the
// energy / force evaluation; metal units: eV, Angstrom, ps, amu).
#include "internal.h"

#include <algorithm>

namespace tsf {

namespace {

// v += c * F / m_type  (c = dt/2 times the unit factor eV/(A amu) -> A/ps^2)
__global__ void k_kick(double *__restrict__ vel, const double *__restrict__ f, const int *__restrict__ types,
                       const double *__restrict__ inv_mass, double c, int n)
{
    const ItemRange r = xcd_items((n + blockDim.x - 1) / blockDim.x);
    for (int it = r.begin; it < r.end; it += r.stride) {
        const int i = it * blockDim.x + threadIdx.x;
        if (i >= n) continue;
        const double w = c * inv_mass[types[i]];
        vel[3 * (size_t)i] += w * f[3 * (size_t)i];
        vel[3 * (size_t)i + 1] += w * f[3 * (size_t)i + 1];
        vel[3 * (size_t)i + 2] += w * f[3 * (size_t)i + 2];
    }
}

// x += dt v
__global__ void k_drift(double *__restrict__ pos, const double *__restrict__ vel, double dt, int n)
{
    const ItemRange r = xcd_items((n + blockDim.x - 1) / blockDim.x);
    for (int it = r.begin; it < r.end; it += r.stride) {
        const int i = it * blockDim.x + threadIdx.x;
        if (i >= n) continue;
        pos[3 * (size_t)i] += dt * vel[3 * (size_t)i];
        pos[3 * (size_t)i + 1] += dt * vel[3 * (size_t)i + 1];
        pos[3 * (size_t)i + 2] += dt * vel[3 * (size_t)i + 2];
    }
}

// *flag = 1 if some atom is farther than sqrt(lim2) from its position at the
// last neighbour build (the list may then miss a pair within the cutoff).
__global__ void k_displaced(const double *__restrict__ pos, const double *__restrict__ pos_build, double lim2,
                            int n, int *flag)
{
    const ItemRange r = xcd_items((n + blockDim.x - 1) / blockDim.x);
    for (int it = r.begin; it < r.end; it += r.stride) {
        const int i = it * blockDim.x + threadIdx.x;
        if (i >= n) continue;
        const double dx = pos[3 * (size_t)i] - pos_build[3 * (size_t)i];
        const double dy = pos[3 * (size_t)i + 1] - pos_build[3 * (size_t)i + 1];
        const double dz = pos[3 * (size_t)i + 2] - pos_build[3 * (size_t)i + 2];
        if (!(dx * dx + dy * dy + dz * dz <= lim2)) atomicOr(flag, 1);
    }
}

// Per-workgroup sums of m v^2 (fixed order within a workgroup).
__global__ void k_kinetic(const double *__restrict__ vel, const int *__restrict__ types,
                          const double *__restrict__ mass, int n, double *__restrict__ partials)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double vx = vel[3 * (size_t)i], vy = vel[3 * (size_t)i + 1], vz = vel[3 * (size_t)i + 2];
        acc += mass[types[i]] * (vx * vx + vy * vy + vz * vz);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

int grid_for(int n) { return std::max(1, std::min((n + 255) / 256, 8192)); }

}  // namespace

hipError_t launch_md_kick(double *vel, const double *f, const int *types, const double *inv_mass, double c, int n,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_kick, dim3(grid_for(n)), dim3(256), 0, s, vel, f, types, inv_mass, c, n);
    return hipGetLastError();
}

hipError_t launch_md_drift(double *pos, const double *vel, double dt, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_drift, dim3(grid_for(n)), dim3(256), 0, s, pos, vel, dt, n);
    return hipGetLastError();
}

hipError_t launch_md_displaced(const double *pos, const double *pos_build, double lim2, int n, int *flag,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_displaced, dim3(grid_for(n)), dim3(256), 0, s, pos, pos_build, lim2, n, flag);
    return hipGetLastError();
}

int md_kinetic_blocks() { return 256; }

hipError_t launch_md_kinetic(const double *vel, const int *types, const double *mass, int n, double *partials,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_kinetic, dim3(md_kinetic_blocks()), dim3(256), 0, s, vel, types, mass, n, partials);
    return hipGetLastError();
}

}  // namespace tsf
