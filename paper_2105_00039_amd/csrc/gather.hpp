// Device building blocks of the 27-box gather (Section IV-A) and of the Eq. 1
// force (Section III), shared by the forward, backward and export kernels.
//
// Agents are stored in box-sorted order, boxes are numbered row-major with x
// fastest, so the 27 boxes around box (ix, iy, iz) are 9 contiguous runs of
// sorted slots: for each (dz, dy) the boxes ix-1 .. ix+1 of one x-row,
// clipped to the grid.  A run is [start[first box], start[last box + 1]).
#pragma once

#include "common.hpp"

namespace ms {

// Fast single-precision square root / reciprocal (about 1 ulp), used on the
// FP32 path whose tolerance is far above their error.
__device__ __forceinline__ float fsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ float frcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double fsqrt(double v) { return sqrt(v); }
__device__ __forceinline__ double frcp(double v) { return 1.0 / v; }

// Simulation of every thread of a block over a sorted or input range:
// thread 0 finds the simulations of the block's first and last index, then
// each thread searches only between them.
__device__ __forceinline__ int block_sim(const int64_t* __restrict__ off, int32_t B, int64_t n,
                                         int64_t first, int64_t i)
{
    __shared__ int s_range[2];
    if (threadIdx.x == 0) {
        const int64_t last = (first + kBlock < n ? first + kBlock : n) - 1;
        s_range[0] = find_sim(off, 0, B, first);
        s_range[1] = find_sim(off, 0, B, last);
    }
    __syncthreads();
    if (i >= n) return 0;
    return find_sim(off, s_range[0], s_range[1] + 1, i);
}

struct Cell { int ix, iy, iz; };

// Box coordinates of a position: the same FP64 binning as the grid build.
template <typename Real>
__device__ __forceinline__ Cell cell_of(const SimGeom& g, Real x, Real y, Real z)
{
    Cell c;
    c.ix = axis_index((double)x, g.origin[0], g.edge, g.dims[0]);
    c.iy = axis_index((double)y, g.origin[1], g.edge, g.dims[1]);
    c.iz = axis_index((double)z, g.origin[2], g.edge, g.dims[2]);
    return c;
}

// Calls fn(j0, j1) for the 9 runs of the 27-box stencil in ascending box
// order ((dz, dy) lexicographic; each run ascending in x).
template <typename Fn>
__device__ __forceinline__ void for_each_run(const SimGeom& g, Cell c, const int32_t* __restrict__ start,
                                             Fn&& fn)
{
    const int nx = g.dims[0], ny = g.dims[1], nz = g.dims[2];
    const int x0 = c.ix > 0 ? c.ix - 1 : 0;
    const int x1 = c.ix + 1 < nx ? c.ix + 1 : nx - 1;
    for (int dz = -1; dz <= 1; ++dz) {
        const int cz = c.iz + dz;
        if (cz < 0 || cz >= nz) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int cy = c.iy + dy;
            if (cy < 0 || cy >= ny) continue;
            const int row = g.box_base + (cz * ny + cy) * nx;
            fn(start[row + x0], start[row + x1 + 1]);
        }
    }
}

// Eq. 1 summed over every candidate in contact with agent `pi`.
// Contact: |u|^2 < (ri + rj)^2, |u| > 0 and delta = ri + rj - |u| > 0.
template <typename Real, typename Pay>
__device__ __forceinline__ void force_sum(const SimGeom& g, Cell c, const Pay& pi,
                                          const int32_t* __restrict__ start,
                                          const Pay* __restrict__ pay, Real kap, Real gam,
                                          Real& fx, Real& fy, Real& fz)
{
    fx = fy = fz = (Real)0;
    Real ax = 0, ay = 0, az = 0;
    for_each_run(g, c, start, [&](int j0, int j1) {
        for (int j = j0; j < j1; ++j) {
            const Pay q = pay[j];
            const Real ux = pi.x - q.x, uy = pi.y - q.y, uz = pi.z - q.z;
            const Real l2 = ux * ux + uy * uy + uz * uz;
            const Real rs = pi.w + q.w;
            if (l2 < rs * rs && l2 > (Real)0) {
                const Real l = fsqrt(l2);
                const Real delta = rs - l;
                if (delta > (Real)0) {
                    const Real rho = pi.w * q.w * frcp(rs);
                    const Real s = kap * delta - gam * fsqrt(rho * delta);
                    const Real sl = s * frcp(l);
                    ax += sl * ux;
                    ay += sl * uy;
                    az += sl * uz;
                }
            }
        }
    });
    fx = ax; fy = ay; fz = az;
}

// Displacement rule (Section III): held if |F| <= adherence, else v = dt F
// bounded in length by max_disp.
template <typename Real>
__device__ __forceinline__ void displacement(Real fx, Real fy, Real fz, Real dt, Real m, Real adh,
                                             Real& dx, Real& dy, Real& dz)
{
    const Real fn = fsqrt(fx * fx + fy * fy + fz * fz);
    if (!(fn > adh)) { dx = dy = dz = (Real)0; return; }
    const Real vx = dt * fx, vy = dt * fy, vz = dt * fz;
    const Real vn = fsqrt(vx * vx + vy * vy + vz * vz);
    if (vn > m) {
        const Real sc = m / vn;
        dx = vx * sc; dy = vy * sc; dz = vz * sc;
    } else {
        dx = vx; dy = vy; dz = vz;
    }
}

}  // namespace ms
