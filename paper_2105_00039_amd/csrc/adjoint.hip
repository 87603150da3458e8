// Reverse-mode derivative of the mechanical step (Eq. 1 and the displacement
// rule of Section III; the paper itself has no backward pass).
//
// Given g_i = dL/dDelta_i:
//   k_bwd_fbar    F_i (kept by the forward step of the same build and
//                 parameters, else recomputed with the forward gather); pull g_i back
//                 through the displacement rule:
//                   |F| <= a : Fbar = 0
//                   |v| <= m : Fbar = dt g
//                   else     : Fbar = dt (m/|v|) (g - vhat (vhat . g))
//                 Fbar is stored in box-sorted order.
//   k_bwd_gather  for every contact (i, j), with e = (p_i - p_j)/l,
//                 w = Fbar_i - Fbar_j, q = e . w,
//                   s_delta = kappa - gamma rho / (2 sqrt(rho delta)),
//                   s_rho   = -gamma delta / (2 sqrt(rho delta)):
//                   pbar_i += (s/l)(w - e q) - s_delta q e
//                   rbar_i += q (s_delta + s_rho r_j^2/(r_i + r_j)^2)
//                   kbar   += delta (e . Fbar_i)
//                   gbar   += -sqrt(rho delta) (e . Fbar_i)
//                 The same 27-box runs as the forward pass; no atomics: every
//                 agent accumulates only its own terms.  kbar and gbar are
//                 summed per block (fixed tree) into one partial per
//                 (block, simulation) pair at index block + simulation.
//   k_reduce_params  one block per simulation sums its partials in a fixed
//                 order, so repeated runs give identical bits.
//
// Rollout mode (ACC): the incoming gradient is dL/dp_{t+1} in the position
// arrays themselves (the state's precision), and the pass turns it into
// dL/dp_t = dL/dp_{t+1} + J^T dL/dp_{t+1} in place, adds the diameter
// gradient to a running sum and the kappa/gamma gradients to running sums:
// one backward step of a rollout p_{t+1} = p_t + Delta(p_t).
#include "gather.hpp"

#include <type_traits>
#include "launch.hpp"

namespace ms {
namespace {

template <int M, bool BATCHED, int LIST>
__global__ __launch_bounds__(kBlock) void k_bwd_fbar(const typename Mode<M>::Pay* __restrict__ pay,
                                                     const int32_t* __restrict__ start,
                                                     const uint32_t* __restrict__ split,
                                                     const int32_t* __restrict__ perm,
                                                     const SimGeom* __restrict__ geom,
                                                     const int64_t* __restrict__ off, int32_t B,
                                                     int64_t n, ms_params p1,
                                                     const ms_params* __restrict__ pB,
                                                     const Header* __restrict__ hdr,
                                                     const typename Mode<M>::Pay* __restrict__ gin,
                                                     typename Mode<M>::Pay* __restrict__ fbar,
                                                     const typename Mode<M>::Pay* __restrict__ fsave,
                                                     const uint2* __restrict__ payq, bool flat)
{
    using Real = typename Mode<M>::Real;
    using Pay = typename Mode<M>::Pay;
    __shared__ uint32_t lst[LIST * kBlock];
    if (hdr->error) return;
    const int64_t k0 = (int64_t)xcd_block() * kBlock;
    const int64_t k = k0 + threadIdx.x;
    int s = 0;
    if (BATCHED) s = block_sim(off, B, n, k0, k, reinterpret_cast<int*>(lst));
    if (k >= n) return;
    const SimGeom g = geom[s];
    const ms_params P = BATCHED ? pB[s] : p1;
    const Pay pi = pay[k];
    const Cell c = cell_of<Real>(g, pi.x, pi.y, pi.z);
    Real fx, fy, fz;
    if (!BATCHED && kept_forces_match(hdr, p1)) {   // uniform: the forward kept F
        const Pay f = fsave[k];
        fx = f.x; fy = f.y; fz = f.z;
    } else {
        force_sum<Real, Pay, LIST>(g, c, pi, (uint32_t)(k * (int64_t)sizeof(Pay)), start, split,
                                        pay, (Real)P.kappa, (Real)P.gamma, lst + threadIdx.x,
                                        preq_of(payq, k), flat, fx, fy, fz);
    }
    const Pay gr = gin[perm[k]];
    const Real gx = gr.x, gy = gr.y, gz = gr.z;
    const Real dt = (Real)P.dt, m = (Real)P.max_disp, a = (Real)P.adherence;
    Pay fb;
    fb.w = (Real)0;
    const Real fn = fsqrt(fx * fx + fy * fy + fz * fz);
    if (!(fn > a)) {
        fb.x = fb.y = fb.z = (Real)0;
    } else {
        const Real vx = dt * fx, vy = dt * fy, vz = dt * fz;
        const Real vn = fsqrt(vx * vx + vy * vy + vz * vz);
        if (vn > m) {
            const Real hx = vx / vn, hy = vy / vn, hz = vz / vn;
            const Real hg = hx * gx + hy * gy + hz * gz;
            const Real sc = dt * (m / vn);
            fb.x = sc * (gx - hx * hg);
            fb.y = sc * (gy - hy * hg);
            fb.z = sc * (gz - hz * hg);
        } else {
            fb.x = dt * gx;
            fb.y = dt * gy;
            fb.z = dt * gz;
        }
    }
    fbar[k] = fb;
}

// The incoming gradient packed into one record per agent (input order), so
// k_bwd_fbar gathers one record per agent instead of three values; and the
// outgoing gradient records split into the caller's arrays.  Both passes are
// coalesced.
template <typename Pay, typename Real, typename G>
__global__ __launch_bounds__(kBlock) void k_pack3(const G* __restrict__ a, const G* __restrict__ b,
                                                  const G* __restrict__ c, int64_t n,
                                                  const Header* __restrict__ hdr, Pay* __restrict__ out)
{
    if (hdr->error) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    Pay v;
    v.x = (Real)a[i]; v.y = (Real)b[i]; v.z = (Real)c[i]; v.w = (Real)0;
    out[i] = v;
}

template <typename Pay, typename Real>
__global__ __launch_bounds__(kBlock) void k_split4(const Pay* __restrict__ in, int64_t n,
                                                   const Header* __restrict__ hdr, Real* __restrict__ a,
                                                   Real* __restrict__ b, Real* __restrict__ c,
                                                   Real* __restrict__ d)
{
    if (hdr->error) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const Pay v = in[i];
    a[i] = v.x; b[i] = v.y; c[i] = v.z; d[i] = v.w;
}

// Rollout mode: pbar += J^T pbar and dbar += (gradient of the diameters),
// in the state's precision In (each term converted first, then added).
template <typename Pay, typename In>
__global__ __launch_bounds__(kBlock) void k_split4_acc(const Pay* __restrict__ in, int64_t n,
                                                       const Header* __restrict__ hdr,
                                                       In* __restrict__ a, In* __restrict__ b,
                                                       In* __restrict__ c, In* __restrict__ d)
{
    if (hdr->error) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const Pay v = in[i];
    a[i] += (In)v.x; b[i] += (In)v.y; c[i] += (In)v.z; d[i] += (In)v.w;
}

// Deterministic block sum: butterfly inside each wave, waves in fixed order.
template <int NT = kBlock>
__device__ __forceinline__ double block_sum_fixed(double v, double* s_w)
{
    v = wave_sum<double>(v);
    if ((threadIdx.x & (kWave - 1)) == 0) s_w[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < NT / kWave; ++w) t += s_w[w];
    __syncthreads();
    return t;
}

// One wavefront per block (NT = kBwdBlock = 64): at 2M agents the backward
// step took 281 -> 273 us at n~12 and 473 -> 446 us at n~30 against
// 256-thread blocks, with four times the kappa/gamma partials.
template <int M, bool BATCHED, int LIST, int NT = kBwdBlock>
__global__ __launch_bounds__(NT) void k_bwd_gather(const typename Mode<M>::Pay* __restrict__ pay,
                                                       const typename Mode<M>::Pay* __restrict__ fbar,
                                                       const int32_t* __restrict__ start,
                                                       const uint32_t* __restrict__ split,
                                                       const int32_t* __restrict__ perm,
                                                       const SimGeom* __restrict__ geom,
                                                       const int64_t* __restrict__ off, int32_t B,
                                                       int64_t n, ms_params p1,
                                                       const ms_params* __restrict__ pB,
                                                       const Header* __restrict__ hdr,
                                                       typename Mode<M>::Pay* __restrict__ gout,
                                                       double* __restrict__ partials,
                                                       const uint2* __restrict__ payq, bool flat)
{
    using Real = typename Mode<M>::Real;
    using Pay = typename Mode<M>::Pay;
    __shared__ double s_w[NT / kWave];
    __shared__ int s_rng[2];
    __shared__ uint32_t lst[LIST * NT];
    if (hdr->error) return;
    const unsigned vb = xcd_block();   // partials are indexed by this virtual block
    const int64_t k0 = (int64_t)vb * NT;
    const int64_t k = k0 + threadIdx.x;
    int s = 0;
    if (BATCHED) {
        s = block_sim<NT>(off, B, n, k0, k, reinterpret_cast<int*>(lst));
        if (threadIdx.x == 0) {
            const int64_t last = (k0 + NT < n ? k0 + NT : n) - 1;
            s_rng[0] = find_sim(off, 0, B, k0);
            s_rng[1] = find_sim(off, 0, B, last);
        }
        __syncthreads();
    }
    double kb = 0.0, gb = 0.0;
    if (k < n) {
        const SimGeom g = geom[s];
        const ms_params P = BATCHED ? pB[s] : p1;
        const Real kap = (Real)P.kappa, gam = (Real)P.gamma;
        const Pay pi = pay[k];
        const Pay fi = fbar[k];
        const Cell c = cell_of<Real>(g, pi.x, pi.y, pi.z);
        const char* fbase = reinterpret_cast<const char*>(fbar);
        Real px = 0, py = 0, pz = 0, rb = 0, kbl = 0, gbl = 0;
        scan_contacts<Real, Pay, LIST, NT>(g, c, pi, (uint32_t)(k * (int64_t)sizeof(Pay)), start,
                                            split, pay, lst + threadIdx.x,
                                            preq_of(payq, k), flat,
                                            [&](uint32_t off, const Pay& q) {
            // loaded before the contact test so a group's loads overlap
            Pay fj = *reinterpret_cast<const Pay*>(fbase + off);
            pin(fj);
            const Real ux = pi.x - q.x, uy = pi.y - q.y, uz = pi.z - q.z;
            const Real l2 = len2(ux, uy, uz);
            const Real rs = pi.w + q.w;
            Real delta, il, rho, sq, h, wj;
            if constexpr (std::is_same<Real, float>::value) {
                // the forward's contact test (same overlap, so the same
                // contacts), and three hardware reciprocal square roots or
                // reciprocals per pair: 1/l, 1/(r_i + r_j), 1/sqrt(rho delta)
                il = __builtin_amdgcn_rsqf(l2);
                delta = fmad(-l2, il, rs);
                if (!(delta > 0.0f)) return;   // coincident centres: NaN delta
                const float ircs = __builtin_amdgcn_rcpf(rs);
                rho = pi.w * q.w * ircs;
                const float rd = rho * delta;
                const float irq = __builtin_amdgcn_rsqf(rd);
                sq = rd * irq;
                h = 0.5f * irq;
                wj = q.w * ircs;
            } else {
                // the forward's FP64 contact decision (correctly rounded |u|)
                // and its refined reciprocals
                const double l = sqrt(l2);
                delta = rs - l;
                if (!(delta > 0.0) || !(l2 > 0.0)) return;
                il = rcp_nr(l);
                const double ircs = rcp_nr(rs);
                rho = pi.w * q.w * ircs;
                const double rd = rho * delta;
                const double irq = rsq_nr(rd);
                sq = rd * irq;
                h = 0.5 * irq;
                wj = q.w * ircs;
            }
            const Real ex = ux * il, ey = uy * il, ez = uz * il;
            const Real sv = kap * delta - gam * sq;
            const Real s_d = kap - gam * rho * h;
            const Real s_r = -gam * delta * h;
            const Real wx = fi.x - fj.x, wy = fi.y - fj.y, wz = fi.z - fj.z;
            const Real qv = ex * wx + ey * wy + ez * wz;
            const Real sl = sv * il;
            px += sl * (wx - ex * qv) - s_d * qv * ex;
            py += sl * (wy - ey * qv) - s_d * qv * ey;
            pz += sl * (wz - ez * qv) - s_d * qv * ez;
            rb += qv * (s_d + s_r * (wj * wj));
            const Real eF = ex * fi.x + ey * fi.y + ez * fi.z;
            kbl += delta * eF;
            gbl -= sq * eF;
        });
        Pay gr;
        gr.x = px;
        gr.y = py;
        gr.z = pz;
        gr.w = (Real)0.5 * rb;
        gout[perm[k]] = gr;
        kb = (double)kbl;
        gb = (double)gbl;
    }
    if (!BATCHED) {
        const double tk = block_sum_fixed<NT>(kb, s_w);
        const double tg = block_sum_fixed<NT>(gb, s_w);
        if (threadIdx.x == 0) {
            partials[2 * vb] = tk;
            partials[2 * vb + 1] = tg;
        }
    } else {
        const int slo = s_rng[0], shi = s_rng[1];
        for (int t = slo; t <= shi; ++t) {
            const bool mine = (k < n) && (s == t);
            const double tk = block_sum_fixed<NT>(mine ? kb : 0.0, s_w);
            const double tg = block_sum_fixed<NT>(mine ? gb : 0.0, s_w);
            if (threadIdx.x == 0) {
                partials[2 * ((int64_t)vb + t)] = tk;
                partials[2 * ((int64_t)vb + t) + 1] = tg;
            }
        }
    }
}

// One block per simulation: sum the partials of the blocks it overlaps.
constexpr int kReduceThreads = 1024;   // threads of the one block per simulation

__global__ __launch_bounds__(kReduceThreads) void k_reduce_params(const double* __restrict__ partials,
                                                          const int64_t* __restrict__ off,
                                                          int64_t n, const Header* __restrict__ hdr,
                                                          double* __restrict__ out, bool acc)
{
    __shared__ double s_w[kReduceThreads / kWave];
    if (hdr->error) return;
    const int s = blockIdx.x;
    const int64_t a0 = off ? off[s] : 0;
    const int64_t a1 = off ? off[s + 1] : n;
    double tk = 0.0, tg = 0.0;
    if (a1 > a0) {
        const int64_t c0 = a0 / kBwdBlock, c1 = (a1 - 1) / kBwdBlock;
        const int64_t sh = off ? s : 0;
        for (int64_t c = c0 + threadIdx.x; c <= c1; c += kReduceThreads) {
            tk += partials[2 * (c + sh)];
            tg += partials[2 * (c + sh) + 1];
        }
    }
    tk = block_sum_fixed<kReduceThreads>(tk, s_w);
    tg = block_sum_fixed<kReduceThreads>(tg, s_w);
    if (threadIdx.x == 0) {
        out[2 * s] = acc ? out[2 * s] + tk : tk;
        out[2 * s + 1] = acc ? out[2 * s + 1] + tg : tg;
    }
}

// acc: rollout mode (gdx..gdz are gx..gz, arrays of the state type In).
template <int M, int LIST>
hipError_t backward_run(const Layout& L, const Dev& D, int64_t n, int32_t B, bool batched,
                        const ms_params* p_host, const ms_params* p_dev, const void* gdx,
                        const void* gdy, const void* gdz, void* gx, void* gy, void* gz, void* gd,
                        double* g_params, bool flat, bool acc, hipStream_t s)
{
    using Real = typename Mode<M>::Real;
    using In = typename Mode<M>::In;
    using Pay = typename Mode<M>::Pay;
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    const unsigned nbg = (unsigned)((n + kBwdBlock - 1) / kBwdBlock);
    const Pay* pay = static_cast<const Pay*>(D.payload);
    Pay* fb = static_cast<Pay*>(D.fbar);
    ms_params dummy{};
    // pay2 (free after the build) holds the packed incoming gradient, then the
    // packed outgoing one
    Pay* rec = static_cast<Pay*>(D.pay2);
    if (acc)
        k_pack3<Pay, Real, In><<<nb, kBlock, 0, s>>>((const In*)gdx, (const In*)gdy, (const In*)gdz,
                                                     n, D.hdr, rec);
    else
        k_pack3<Pay, Real, Real><<<nb, kBlock, 0, s>>>((const Real*)gdx, (const Real*)gdy,
                                                       (const Real*)gdz, n, D.hdr, rec);
    if (batched) {
        k_bwd_fbar<M, true, LIST><<<nb, kBlock, 0, s>>>(pay, D.start, D.split, D.perm, D.geom, D.off, B, n,
                                                   dummy, p_dev, D.hdr, rec, fb, nullptr, D.payq,
                                                   flat);
        k_bwd_gather<M, true, LIST><<<nbg, kBwdBlock, 0, s>>>(pay, fb, D.start, D.split, D.perm, D.geom, D.off, B,
                                                     n, dummy, p_dev, D.hdr, rec, D.partials, D.payq,
                                                     flat);
        k_reduce_params<<<B, kReduceThreads, 0, s>>>(D.partials, D.off, n, D.hdr, g_params, acc);
    } else {
        k_bwd_fbar<M, false, LIST><<<nb, kBlock, 0, s>>>(pay, D.start, D.split, D.perm, D.geom, nullptr, 1,
                                                    n, *p_host, nullptr, D.hdr, rec, fb,
                                                    static_cast<const Pay*>(D.fsave), D.payq, flat);
        k_bwd_gather<M, false, LIST><<<nbg, kBwdBlock, 0, s>>>(pay, fb, D.start, D.split, D.perm, D.geom, nullptr,
                                                      1, n, *p_host, nullptr, D.hdr, rec,
                                                      D.partials, D.payq, flat);
        k_reduce_params<<<1, kReduceThreads, 0, s>>>(D.partials, nullptr, n, D.hdr, g_params, acc);
    }
    if (acc)
        k_split4_acc<Pay, In><<<nb, kBlock, 0, s>>>(rec, n, D.hdr, (In*)gx, (In*)gy, (In*)gz, (In*)gd);
    else
        k_split4<Pay, Real><<<nb, kBlock, 0, s>>>(rec, n, D.hdr, (Real*)gx, (Real*)gy, (Real*)gz,
                                                  (Real*)gd);
    return hipGetLastError();
}

// list: contact-list length of the gathers (the workspace's choice for the
// forward step; results do not depend on it).
template <int M>
hipError_t backward_mode(const Layout& L, const Dev& D, int64_t n, int32_t B, bool batched,
                         const ms_params* p_host, const ms_params* p_dev, const void* gdx,
                         const void* gdy, const void* gdz, void* gx, void* gy, void* gz, void* gd,
                         double* g_params, int list, bool flat, bool acc, hipStream_t s)
{
    if (list == kLongList)
        return backward_run<M, kLongList>(L, D, n, B, batched, p_host, p_dev, gdx, gdy, gdz, gx, gy,
                                          gz, gd, g_params, flat, acc, s);
    return backward_run<M, kMaxContacts>(L, D, n, B, batched, p_host, p_dev, gdx, gdy, gdz, gx, gy,
                                         gz, gd, g_params, flat, acc, s);
}

}  // namespace

hipError_t launch_backward(const Layout& L, const Dev& D, int64_t n, int32_t B, bool batched,
                           const ms_params* p_host, const ms_params* p_dev, const void* gdx,
                           const void* gdy, const void* gdz, void* gx, void* gy, void* gz,
                           void* gd, double* g_params, int list, bool flat, bool acc,
                           hipStream_t s)
{
    switch (L.dtype) {
    case MS_F32:
        return backward_mode<MS_F32>(L, D, n, B, batched, p_host, p_dev, gdx, gdy, gdz, gx, gy, gz,
                                     gd, g_params, list, flat, acc, s);
    case MS_F64:
        return backward_mode<MS_F64>(L, D, n, B, batched, p_host, p_dev, gdx, gdy, gdz, gx, gy, gz,
                                     gd, g_params, list, flat, acc, s);
    case MS_F32_POS64:
        return backward_mode<MS_F32_POS64>(L, D, n, B, batched, p_host, p_dev, gdx, gdy, gdz, gx,
                                           gy, gz, gd, g_params, list, flat, acc, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ms
