// Forward mechanical step (Section III, Eq. 1 and the displacement rule),
// position update, neighbour-set export and the bandwidth probe.
//
// k_force: one lane per agent in box-sorted order (the paper's GPU kernels
// also give each thread one agent).  Consecutive lanes hold agents of the same
// or neighbouring boxes, so a wavefront walks nearly the same 9 runs and its
// candidate loads are served by L1/L2.  The force is summed in registers in
// ascending (box, quarter, input index) order; the displacement is stored at
// the agent's input position through perm (as one record, split by k_soa).
// In the sorted-state step (SORTED) the kernel instead writes the agent's
// position after the step and its diameter at its own slot, so every store
// is coalesced and no split pass follows: the state comes out renumbered in
// the build's slot order (the agent sorting of Section IV-D, kept across a
// rollout).
#include "gather.hpp"
#include "launch.hpp"

namespace ms {
namespace {

// Outputs of the sorted-state step, all in slot order: the state after the
// step (positions and diameters of the caller's type In) and, when dx is
// non-null, the displacements (Real).  xi..di: the build's inputs, read
// (through perm) only where the payload does not hold them exactly, i.e. the
// FP64 master positions and diameters of MS_F32_POS64.
template <typename In, typename Real>
struct SortedOut {
    In *x, *y, *z, *d;
    Real *dx, *dy, *dz;
    const In *xi, *yi, *zi, *di;
};

// Plain FP64 builds ask for at least 4 wavefronts per SIMD (at most 128
// VGPRs, against 131 otherwise): with 3 the gather's loads are hidden worse
// (force kernel at 2M agents, n~12: 309 -> 287 us).
template <int M, bool BATCHED, int LIST, bool SORTED, int NT>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(M == MS_F64 && !BATCHED ? 4 : 1))) void k_force(const typename Mode<M>::Pay* __restrict__ pay,
                                                  const int32_t* __restrict__ start,
                                                  const uint32_t* __restrict__ split,
                                                  const int32_t* __restrict__ perm,
                                                  const SimGeom* __restrict__ geom,
                                                  const int64_t* __restrict__ off, int32_t B,
                                                  int64_t n, ms_params p1,
                                                  const ms_params* __restrict__ pB,
                                                  Header* __restrict__ hdr,
                                                  typename Mode<M>::Pay* __restrict__ dout,
                                                  typename Mode<M>::Pay* __restrict__ fsave,
                                                  const uint2* __restrict__ payq,
                                                  SortedOut<typename Mode<M>::In, typename Mode<M>::Real> so,
                                                  bool flat)
{
    using Real = typename Mode<M>::Real;
    using In = typename Mode<M>::In;
    using Pay = typename Mode<M>::Pay;
    __shared__ uint32_t lst[LIST * NT];
    if (hdr->error) return;
    // forces kept for the backward step: record which build and parameters
    // they belong to (the backward uses them only on a match)
    if (fsave && blockIdx.x == 0 && threadIdx.x == 0) {
        hdr->fwd_gen = hdr->build_gen;
        hdr->fwd_params = p1;
    }
    const int64_t k0 = (int64_t)xcd_block() * NT;
    const int64_t k = k0 + threadIdx.x;
    int s = 0;
    if (BATCHED) s = block_sim<NT>(off, B, n, k0, k, reinterpret_cast<int*>(lst));
    if (k >= n) return;
    const SimGeom g = geom[s];
    const ms_params P = BATCHED ? pB[s] : p1;
    const Pay pi = pay[k];
    // sorted-state step of FP64 positions: the master state of this slot is
    // read through perm, issued here so its latency hides behind the gather
    In mx = 0, my = 0, mz = 0, md = 0;
    if constexpr (SORTED && M == MS_F32_POS64) {
        const int32_t o = perm[k];
        mx = so.xi[o]; my = so.yi[o]; mz = so.zi[o]; md = so.di[o];
    }
    const Cell c = cell_of<Real>(g, pi.x, pi.y, pi.z);
    Real fx, fy, fz;
    force_sum<Real, Pay, LIST, NT>(g, c, pi, (uint32_t)(k * (int64_t)sizeof(Pay)), start, split,
                                    pay, (Real)P.kappa, (Real)P.gamma, lst + threadIdx.x,
                                    preq_of(payq, k), flat, fx, fy, fz);
    if (fsave) {
        Pay f;
        f.x = fx; f.y = fy; f.z = fz; f.w = (Real)0;
        fsave[k] = f;
    }
    Real ddx, ddy, ddz;
    displacement<Real>(fx, fy, fz, (Real)P.dt, (Real)P.max_disp, (Real)P.adherence, ddx, ddy, ddz);
    if constexpr (SORTED) {
        // p + Delta as k_soa_integrate forms it (Delta converted to In, then
        // added): the step equals the caller-order step renumbered
        In px, py, pz, pd;
        if constexpr (M == MS_F32_POS64) {
            px = mx; py = my; pz = mz; pd = md;
        } else {
            px = pi.x; py = pi.y; pz = pi.z;
            pd = (In)2 * pi.w;   // the build stored d/2: exact for every normal d
        }
        so.x[k] = px + (In)ddx;
        so.y[k] = py + (In)ddy;
        so.z[k] = pz + (In)ddz;
        so.d[k] = pd;
        if (so.dx) { so.dx[k] = ddx; so.dy[k] = ddy; so.dz[k] = ddz; }
    } else {
        const int32_t o = perm[k];
        Pay v;
        v.x = ddx; v.y = ddy; v.z = ddz; v.w = (Real)0;
        dout[o] = v;
    }
}

// The force kernel stores each displacement as one 16-byte (FP64: 32-byte)
// record at the agent's input position: one random store instead of three
// 4-byte ones, each of which costs a whole DRAM sector.  This pass splits the
// records into the caller's dx, dy, dz with coalesced accesses.
template <typename Pay, typename Real>
__global__ __launch_bounds__(kBlock) void k_soa(const Pay* __restrict__ a, int64_t n,
                                                const Header* __restrict__ hdr,
                                                Real* __restrict__ dx, Real* __restrict__ dy,
                                                Real* __restrict__ dz)
{
    if (hdr->error) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const Pay v = a[i];
    dx[i] = v.x; dy[i] = v.y; dz[i] = v.z;
}

// k_soa fused with the position update of a rollout: p += Delta in place
// (p in the caller's order, Delta converted as k_integrate converts it), and
// Delta itself written when dx is non-null.  Nothing moves after a device
// error.
template <typename Pay, typename Real, typename PT>
__global__ __launch_bounds__(kBlock) void k_soa_integrate(const Pay* __restrict__ a, int64_t n,
                                                          const Header* __restrict__ hdr,
                                                          Real* __restrict__ dx, Real* __restrict__ dy,
                                                          Real* __restrict__ dz, PT* __restrict__ x,
                                                          PT* __restrict__ y, PT* __restrict__ z)
{
    if (hdr->error) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const Pay v = a[i];
    if (dx) { dx[i] = v.x; dy[i] = v.y; dz[i] = v.z; }
    x[i] += (PT)v.x;
    y[i] += (PT)v.y;
    z[i] += (PT)v.z;
}

template <typename PT, typename DT>
__global__ __launch_bounds__(kBlock) void k_integrate(PT* __restrict__ x, PT* __restrict__ y,
                                                      PT* __restrict__ z,
                                                      const DT* __restrict__ dx,
                                                      const DT* __restrict__ dy,
                                                      const DT* __restrict__ dz, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    x[i] += (PT)dx[i];
    y[i] += (PT)dy[i];
    z[i] += (PT)dz[i];
}

// Neighbour sets with the FP64 predicate |p_j - p_i|^2 < edge^2, the square
// evaluated as (ux*ux + uy*uy) + uz*uz with no fused multiply-add so that it
// is reproducible bit for bit.  Candidates are visited in canonical order
// (ascending box, then input index) through cslot, the payload slot of each
// canonical slot; list entries are input indices (canon).
template <int M, bool BATCHED, bool FILL>
__global__ __launch_bounds__(kBlock) void k_neighbors(const typename Mode<M>::Pay* __restrict__ pay,
                                                      const int32_t* __restrict__ start,
                                                      const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ canon,
                                                      const int32_t* __restrict__ cslot,
                                                      const SimGeom* __restrict__ geom,
                                                      const int64_t* __restrict__ off, int32_t B,
                                                      int64_t n, const Header* __restrict__ hdr,
                                                      int32_t* __restrict__ counts,
                                                      const int64_t* __restrict__ offsets,
                                                      int32_t* __restrict__ list)
{
#pragma clang fp contract(off)
    using Real = typename Mode<M>::Real;
    using Pay = typename Mode<M>::Pay;
    if (hdr->error) return;
    const int64_t k0 = (int64_t)xcd_block() * kBlock;
    const int64_t k = k0 + threadIdx.x;
    __shared__ int s_range[2];
    int s = 0;
    if (BATCHED) s = block_sim(off, B, n, k0, k, s_range);
    if (k >= n) return;
    const SimGeom g = geom[s];
    const Pay pi = pay[k];
    const Cell c = cell_of<Real>(g, pi.x, pi.y, pi.z);
    const double xi = (double)pi.x, yi = (double)pi.y, zi = (double)pi.z;
    const double e2 = g.edge * g.edge;
    const int32_t me = perm[k];
    int64_t cnt = 0;
    const int64_t base = FILL ? offsets[me] : 0;
    for_each_run(g, c, start, [&](int j0, int j1) {
        for (int cc = j0; cc < j1; ++cc) {
            const int j = cslot[cc];
            if (j == (int)k) continue;
            const Pay q = pay[j];
            const double ux = (double)q.x - xi, uy = (double)q.y - yi, uz = (double)q.z - zi;
            const double d2 = (ux * ux + uy * uy) + uz * uz;
            if (d2 < e2) {
                if (FILL) list[base + cnt] = canon[cc];
                ++cnt;
            }
        }
    });
    if (!FILL) counts[me] = (int32_t)cnt;
}

// Three-phase exclusive scan of int32 counts [n] into int64 offsets [n+1].
__global__ __launch_bounds__(kBlock) void k_tile_sums(const int32_t* __restrict__ in, int64_t n,
                                                      long long* __restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    long long v = 0;
    for (int k = threadIdx.x; k < kScanTile; k += kBlock) {
        const int64_t i = base + k;
        if (i < n) v += in[i];
    }
    v = wave_sum<long long>(v);
    __shared__ long long s_w[kBlock / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) s_w[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += s_w[w];
        sums[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_sums(long long* sums, int64_t ntiles)
{
    // single block, sequential over chunks of kBlock tiles
    __shared__ long long s_v[kBlock];
    long long running = 0;
    for (int64_t c = 0; c < ntiles; c += kBlock) {
        const int64_t t = c + threadIdx.x;
        const long long v = t < ntiles ? sums[t] : 0;
        s_v[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kBlock; o <<= 1) {
            long long a = threadIdx.x >= (unsigned)o ? s_v[threadIdx.x - o] : 0;
            __syncthreads();
            s_v[threadIdx.x] += a;
            __syncthreads();
        }
        const long long inc = s_v[threadIdx.x];
        const long long tot = s_v[kBlock - 1];
        if (t < ntiles) sums[t] = running + inc - v;
        running += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[ntiles] = running;
}

__global__ __launch_bounds__(kBlock) void k_tile_scan(const int32_t* __restrict__ in, int64_t n,
                                                      const long long* __restrict__ sums,
                                                      int64_t* __restrict__ out)
{
    __shared__ long long s_v[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    long long v[kScanItems];
    long long tsum = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        v[k] = i < n ? in[i] : 0;
        tsum += v[k];
    }
    s_v[threadIdx.x] = tsum;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        long long a = threadIdx.x >= (unsigned)o ? s_v[threadIdx.x - o] : 0;
        __syncthreads();
        s_v[threadIdx.x] += a;
        __syncthreads();
    }
    long long run = sums[blockIdx.x] + s_v[threadIdx.x] - tsum;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        if (i <= n) out[i] = run;
        run += v[k];
    }
}

__global__ __launch_bounds__(kBlock) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                 int64_t n4)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n4; i += stride) dst[i] = src[i];
}

template <int M, bool BATCHED, int LIST, bool SORTED, int NT>
void launch_k_force(const Dev& D, int64_t n, int32_t B, const ms_params& p1, const ms_params* p_dev,
                    typename Mode<M>::Pay* rec, typename Mode<M>::Pay* fs,
                    const SortedOut<typename Mode<M>::In, typename Mode<M>::Real>& so, bool flat,
                    hipStream_t s)
{
    using Pay = typename Mode<M>::Pay;
    const unsigned nb = (unsigned)((n + NT - 1) / NT);
    k_force<M, BATCHED, LIST, SORTED, NT><<<nb, NT, 0, s>>>(
        static_cast<const Pay*>(D.payload), D.start, D.split, D.perm, D.geom, BATCHED ? D.off : nullptr,
        B, n, p1, p_dev, D.hdr, rec, fs, D.payq, so, flat);
}

template <int M, bool BATCHED, bool SORTED, int NT>
void launch_k_force_nt(const Dev& D, int64_t n, int32_t B, const ms_params& p1,
                       const ms_params* p_dev, typename Mode<M>::Pay* rec,
                       typename Mode<M>::Pay* fs,
                       const SortedOut<typename Mode<M>::In, typename Mode<M>::Real>& so, int list,
                       bool flat, hipStream_t s)
{
    if (list == kLongList)
        launch_k_force<M, BATCHED, kLongList, SORTED, NT>(D, n, B, p1, p_dev, rec, fs, so, flat, s);
    else
        launch_k_force<M, BATCHED, kMaxContacts, SORTED, NT>(D, n, B, p1, p_dev, rec, fs, so, flat,
                                                              s);
}

// The forward gather's launch shape chosen per workspace: contact-list length
// (kMaxContacts or kLongList) and threads per block (kForceBlockSmall or kBlock).
template <int M, bool SORTED>
void launch_k_force_list(const Dev& D, int64_t n, int32_t B, bool batched, const ms_params& p1,
                         const ms_params* p_dev, typename Mode<M>::Pay* rec,
                         typename Mode<M>::Pay* fs,
                         const SortedOut<typename Mode<M>::In, typename Mode<M>::Real>& so, int list,
                         int nt, bool flat, hipStream_t s)
{
    if (batched && nt == kForceBlockSmall)
        launch_k_force_nt<M, true, SORTED, kForceBlockSmall>(D, n, B, p1, p_dev, rec, nullptr, so,
                                                             list, flat, s);
    else if (batched)
        launch_k_force_nt<M, true, SORTED, kBlock>(D, n, B, p1, p_dev, rec, nullptr, so, list,
                                                   flat, s);
    else if (nt == kForceBlockSmall)
        launch_k_force_nt<M, false, SORTED, kForceBlockSmall>(D, n, 1, p1, nullptr, rec, fs, so,
                                                              list, flat, s);
    else
        launch_k_force_nt<M, false, SORTED, kBlock>(D, n, 1, p1, nullptr, rec, fs, so, list, flat,
                                                    s);
}

template <int M>
hipError_t force_mode(const Layout& L, const Dev& D, int64_t n, int32_t B, bool batched,
                      const ms_params* p_host, const ms_params* p_dev, void* dx, void* dy,
                      void* dz, void* px, void* py, void* pz, bool keep, int list, int nt,
                      bool flat, const SortedState* sorted, hipStream_t s)
{
    using Real = typename Mode<M>::Real;
    using In = typename Mode<M>::In;
    using Pay = typename Mode<M>::Pay;
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    Real* X = static_cast<Real*>(dx);
    Real* Y = static_cast<Real*>(dy);
    Real* Z = static_cast<Real*>(dz);
    Pay* A = static_cast<Pay*>(D.pay2);
    Pay* fs = (keep && !batched) ? static_cast<Pay*>(D.fsave) : nullptr;
    const ms_params p1 = batched ? ms_params{} : *p_host;
    SortedOut<In, Real> so{};
    if (sorted) {
        so.x = static_cast<In*>(sorted->x_out); so.y = static_cast<In*>(sorted->y_out);
        so.z = static_cast<In*>(sorted->z_out); so.d = static_cast<In*>(sorted->d_out);
        so.dx = X; so.dy = Y; so.dz = Z;
        so.xi = static_cast<const In*>(sorted->x_in); so.yi = static_cast<const In*>(sorted->y_in);
        so.zi = static_cast<const In*>(sorted->z_in); so.di = static_cast<const In*>(sorted->d_in);
        launch_k_force_list<M, true>(D, n, B, batched, p1, p_dev, A, fs, so, list, nt, flat, s);
        return hipGetLastError();
    }
    launch_k_force_list<M, false>(D, n, B, batched, p1, p_dev, A, fs, so, list, nt, flat, s);
    if (px) {
        k_soa_integrate<Pay, Real, In><<<nb, kBlock, 0, s>>>(A, n, D.hdr, X, Y, Z, static_cast<In*>(px),
                                                             static_cast<In*>(py),
                                                             static_cast<In*>(pz));
    } else {
        k_soa<Pay, Real><<<nb, kBlock, 0, s>>>(A, n, D.hdr, X, Y, Z);
    }
    return hipGetLastError();
}

template <int M>
hipError_t nbr_mode(const Layout& L, const Dev& D, int64_t n, int32_t B, bool batched,
                    int32_t* counts, int64_t* offsets, int32_t* list, bool fill, hipStream_t s)
{
    using Pay = typename Mode<M>::Pay;
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    const Pay* pay = static_cast<const Pay*>(D.payload);
    const int64_t* off = batched ? D.off : nullptr;
    if (!fill) {
        if (batched)
            k_neighbors<M, true, false><<<nb, kBlock, 0, s>>>(pay, D.start, D.perm, D.canon, D.cslot,
                                                               D.geom, off, B,
                                                               n, D.hdr, counts, nullptr, nullptr);
        else
            k_neighbors<M, false, false><<<nb, kBlock, 0, s>>>(pay, D.start, D.perm, D.canon, D.cslot,
                                                                D.geom, off, 1,
                                                                n, D.hdr, counts, nullptr, nullptr);
        const int64_t ntiles = (n + 1 + kScanTile - 1) / kScanTile;
        k_tile_sums<<<(unsigned)ntiles, kBlock, 0, s>>>(counts, n, D.scratch64);
        k_scan_sums<<<1, kBlock, 0, s>>>(D.scratch64, ntiles);
        k_tile_scan<<<(unsigned)ntiles, kBlock, 0, s>>>(counts, n, D.scratch64, offsets);
    } else {
        if (batched)
            k_neighbors<M, true, true><<<nb, kBlock, 0, s>>>(pay, D.start, D.perm, D.canon, D.cslot,
                                                              D.geom, off, B, n,
                                                              D.hdr, nullptr, offsets, list);
        else
            k_neighbors<M, false, true><<<nb, kBlock, 0, s>>>(pay, D.start, D.perm, D.canon, D.cslot,
                                                               D.geom, off, 1,
                                                               n, D.hdr, nullptr, offsets, list);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_force(const Layout& L, const Dev& D, int64_t n, int32_t B, bool batched,
                        const ms_params* p_host, const ms_params* p_dev, void* dx, void* dy,
                        void* dz, void* px, void* py, void* pz, bool keep, int list, int nt,
                        bool flat, hipStream_t s, const SortedState* sorted)
{
    switch (L.dtype) {
    case MS_F32:
        return force_mode<MS_F32>(L, D, n, B, batched, p_host, p_dev, dx, dy, dz, px, py, pz, keep,
                                  list, nt, flat, sorted, s);
    case MS_F64:
        return force_mode<MS_F64>(L, D, n, B, batched, p_host, p_dev, dx, dy, dz, px, py, pz, keep,
                                  list, nt, flat, sorted, s);
    case MS_F32_POS64:
        return force_mode<MS_F32_POS64>(L, D, n, B, batched, p_host, p_dev, dx, dy, dz, px, py, pz,
                                        keep, list, nt, flat, sorted, s);
    default: return hipErrorInvalidValue;
    }
}

// dst[k] = src[perm[k]]: any per-agent array into the slot order of the
// last build.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_reorder(const int32_t* __restrict__ perm,
                                                    const T* __restrict__ src, T* __restrict__ dst,
                                                    int64_t n, const Header* __restrict__ hdr)
{
    if (hdr->error) return;
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < n) dst[k] = src[perm[k]];
}

hipError_t launch_reorder(const Dev& D, int64_t n, const void* src, void* dst, int elem_bytes,
                          hipStream_t s)
{
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    switch (elem_bytes) {
    case 1: k_reorder<uint8_t><<<nb, kBlock, 0, s>>>(D.perm, (const uint8_t*)src, (uint8_t*)dst, n, D.hdr); break;
    case 2: k_reorder<uint16_t><<<nb, kBlock, 0, s>>>(D.perm, (const uint16_t*)src, (uint16_t*)dst, n, D.hdr); break;
    case 4: k_reorder<uint32_t><<<nb, kBlock, 0, s>>>(D.perm, (const uint32_t*)src, (uint32_t*)dst, n, D.hdr); break;
    case 8: k_reorder<uint2><<<nb, kBlock, 0, s>>>(D.perm, (const uint2*)src, (uint2*)dst, n, D.hdr); break;
    case 16: k_reorder<uint4><<<nb, kBlock, 0, s>>>(D.perm, (const uint4*)src, (uint4*)dst, n, D.hdr); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_integrate(void* x, void* y, void* z, const void* dx, const void* dy,
                            const void* dz, int64_t n, int dtype, hipStream_t s)
{
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    switch (dtype) {
    case MS_F32:
        k_integrate<float, float><<<nb, kBlock, 0, s>>>(
            (float*)x, (float*)y, (float*)z, (const float*)dx, (const float*)dy, (const float*)dz, n);
        break;
    case MS_F64:
        k_integrate<double, double><<<nb, kBlock, 0, s>>>((double*)x, (double*)y, (double*)z,
                                                          (const double*)dx, (const double*)dy,
                                                          (const double*)dz, n);
        break;
    case MS_F32_POS64:
        k_integrate<double, float><<<nb, kBlock, 0, s>>>((double*)x, (double*)y, (double*)z,
                                                         (const float*)dx, (const float*)dy,
                                                         (const float*)dz, n);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_neighbors_count(const Layout& L, const Dev& D, int64_t n, int32_t B, bool batched,
                                  int32_t* counts, int64_t* offsets, hipStream_t s)
{
    switch (L.dtype) {
    case MS_F32: return nbr_mode<MS_F32>(L, D, n, B, batched, counts, offsets, nullptr, false, s);
    case MS_F64: return nbr_mode<MS_F64>(L, D, n, B, batched, counts, offsets, nullptr, false, s);
    case MS_F32_POS64:
        return nbr_mode<MS_F32_POS64>(L, D, n, B, batched, counts, offsets, nullptr, false, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_neighbors_fill(const Layout& L, const Dev& D, int64_t n, int32_t B, bool batched,
                                 const int64_t* offsets, int32_t* list, hipStream_t s)
{
    int64_t* o = const_cast<int64_t*>(offsets);
    switch (L.dtype) {
    case MS_F32: return nbr_mode<MS_F32>(L, D, n, B, batched, nullptr, o, list, true, s);
    case MS_F64: return nbr_mode<MS_F64>(L, D, n, B, batched, nullptr, o, list, true, s);
    case MS_F32_POS64:
        return nbr_mode<MS_F32_POS64>(L, D, n, B, batched, nullptr, o, list, true, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_copy_probe(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    const int64_t n4 = (int64_t)(bytes / 16);
    int64_t blocks = (n4 + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    k_copy<<<(unsigned)blocks, kBlock, 0, s>>>(static_cast<const uint4*>(src),
                                                static_cast<uint4*>(dst), n4);
    return hipGetLastError();
}

}  // namespace ms
