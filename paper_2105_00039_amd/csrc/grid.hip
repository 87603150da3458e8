// Uniform-grid construction on the device (Section IV-A of the paper: a
// regular grid of boxes rebuilt every timestep; each box knows its agents).
//
// The paper keeps, per box, a count and the last agent added, and links the
// agents of a box through a successor list.  Here the same information is a
// counting sort held in the workspace:
//   k_bounds    per-simulation min/max of x, y, z and max diameter
//               (block reduction, then one 64-bit atomic per value and block on
//               an order-preserving integer encoding)
//   k_geometry  edge, origin, dims, number of boxes, global box base of every
//               simulation (one block), error word, scan epoch
//   k_count     global box index per agent (FP64 binning) and an arrival slot
//               from an atomic increment of the box count
//   k_scan      exclusive scan of the counts -> box start offsets
//               (single pass, decoupled look-back; zeroes the counts it reads so
//               the next build starts from zero)
//   k_scatter   agent index into its arrival slot
//   k_rank      final slot = box start + number of box mates with a smaller
//               input index (stable order), plus the sorted copy of
//               (x, y, z, d/2) used by the force gather
#include "launch.hpp"

namespace ms {
namespace {

constexpr uint32_t ERR_OFFSETS = 16u;   // sim offsets not a valid partition of [0, n)

// ----------------------------------------------------------------- helpers

template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* s_wave, T& total)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    T x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) s_wave[wid] = x;
    __syncthreads();
    T wp = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        T t = s_wave[w];
        if (w < wid) wp += t;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return wp + x - v;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}

// ------------------------------------------------------------------- init

__global__ void k_init(Header* hdr, SimAcc* acc, int32_t max_sims, int32_t* count, int64_t ncount,
                       unsigned long long* flags, int64_t nflags)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t; i < ncount; i += stride) count[i] = 0;
    for (int64_t i = t; i < nflags; i += stride) flags[i] = 0ull;
    for (int64_t s = t; s < max_sims; s += stride) {
        SimAcc a;
        for (int k = 0; k < 3; ++k) { a.lo[k] = ~0ull; a.hi[k] = 0ull; }
        a.dmax = 0ull;
        a.flags = 0ull;
        acc[s] = a;
    }
    if (t < (int64_t)(sizeof(Header) / 4)) reinterpret_cast<uint32_t*>(hdr)[t] = 0u;
}

// ------------------------------------------------------------- offsets copy

// Copies the caller's simulation offsets into the workspace and checks that
// they partition [0, n).
__global__ void k_copy_offsets(const int64_t* __restrict__ in, int64_t* out, int32_t B, int64_t n,
                               SimAcc* acc)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > B) return;
    const int64_t v = in[s];
    out[s] = v;
    bool bad = (v < 0) || (v > n) || (s == 0 && v != 0) || (s == B && v != n);
    if (s < B && in[s + 1] < v) bad = true;
    if (bad) atomicOr(&acc[0].flags, (unsigned long long)ERR_OFFSETS);
}

// ------------------------------------------------------------------ bounds

template <int M, bool BATCHED>
__global__ __launch_bounds__(kBlock) void k_bounds(const typename Mode<M>::In* __restrict__ x,
                                                   const typename Mode<M>::In* __restrict__ y,
                                                   const typename Mode<M>::In* __restrict__ z,
                                                   const typename Mode<M>::In* __restrict__ d,
                                                   int64_t n, const int64_t* __restrict__ off,
                                                   int32_t B, SimAcc* acc)
{
    using Real = typename Mode<M>::Real;
    __shared__ int s_range[2];
    __shared__ double s_red[7][kBlock / kWave];
    __shared__ uint32_t s_flag[kBlock / kWave];
    const int64_t c0 = (int64_t)blockIdx.x * kBoundsChunk;
    const int64_t c1 = (c0 + kBoundsChunk < n) ? c0 + kBoundsChunk : n;
    int slo = 0, shi = 0;
    if (BATCHED) {
        if (threadIdx.x == 0) {
            s_range[0] = find_sim(off, 0, B, c0);
            s_range[1] = find_sim(off, 0, B, c1 - 1);
        }
        __syncthreads();
        slo = s_range[0];
        shi = s_range[1];
    }
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    for (int s = slo; s <= shi; ++s) {
        int64_t a0 = c0, a1 = c1;
        if (BATCHED) {
            a0 = off[s] > c0 ? off[s] : c0;
            a1 = off[s + 1] < c1 ? off[s + 1] : c1;
        }
        if (a1 <= a0) continue;   // block-uniform
        double lo[3] = {INFINITY, INFINITY, INFINITY};
        double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double dm = -INFINITY;
        uint32_t fl = 0;
        for (int64_t i = a0 + threadIdx.x; i < a1; i += kBlock) {
            const double p[3] = {(double)(Real)x[i], (double)(Real)y[i], (double)(Real)z[i]};
            const double di = (double)(Real)d[i];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (!isfinite(p[k])) fl |= ERR_NONFINITE;
                lo[k] = fmin(lo[k], p[k]);
                hi[k] = fmax(hi[k], p[k]);
            }
            if (!isfinite(di)) fl |= ERR_NONFINITE;
            if (di < 0.0) fl |= ERR_NEGDIAM;
            dm = fmax(dm, di);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = wave_min(lo[k]);
            hi[k] = wave_max(hi[k]);
        }
        dm = wave_max(dm);
        fl = wave_or(fl);
        if (lane == 0) {
            for (int k = 0; k < 3; ++k) { s_red[k][wid] = lo[k]; s_red[3 + k][wid] = hi[k]; }
            s_red[6][wid] = dm;
            s_flag[wid] = fl;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < kBlock / kWave; ++w) {
                for (int k = 0; k < 3; ++k) {
                    lo[k] = fmin(lo[k], s_red[k][w]);
                    hi[k] = fmax(hi[k], s_red[3 + k][w]);
                }
                dm = fmax(dm, s_red[6][w]);
                fl |= s_flag[w];
            }
            SimAcc* A = acc + s;
            for (int k = 0; k < 3; ++k) {
                atomicMin(&A->lo[k], enc_f64(lo[k]));
                atomicMax(&A->hi[k], enc_f64(hi[k]));
            }
            atomicMax(&A->dmax, enc_f64(dm));
            if (fl) atomicOr(&A->flags, (unsigned long long)fl);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- geometry

// One block.  Reads and resets the accumulators, fixes each simulation's
// edge (caller's, or its largest diameter), origin (minimum), dims
// (floor((max - min)/edge) + 1) and box range, and rewrites the error word.
__global__ __launch_bounds__(kBlock) void k_geometry(Header* hdr, SimAcc* acc, SimGeom* geom,
                                                     const int64_t* __restrict__ off, int64_t n,
                                                     int32_t B, double edge,
                                                     const double* __restrict__ edges,
                                                     int64_t max_boxes)
{
    __shared__ long long s_wave[kBlock / kWave];
    __shared__ uint32_t s_err;
    if (threadIdx.x == 0) s_err = 0;
    __syncthreads();
    long long running = 0;
    for (int c = 0; c < B; c += kBlock) {
        const int s = c + threadIdx.x;
        long long nb = 0;
        uint32_t err = 0;
        SimGeom g{};
        if (s < B) {
            SimAcc a = acc[s];
            SimAcc r;
            for (int k = 0; k < 3; ++k) { r.lo[k] = ~0ull; r.hi[k] = 0ull; }
            r.dmax = 0ull;
            r.flags = 0ull;
            acc[s] = r;
            err = (uint32_t)a.flags;
            const int64_t ns = off ? off[s + 1] - off[s] : n;
            double e = edges ? edges[s] : edge;
            const double dmax = dec_f64(a.dmax);
            if (!isfinite(e)) err |= ERR_EDGE;
            else if (e <= 0.0) e = dmax;
            g.edge = e;
            if (ns > 0 && err == 0) {
                if (!(e > 0.0) || e < dmax) err |= ERR_EDGE;
            }
            if (ns > 0 && err == 0) {
                long long prod = 1;
                for (int k = 0; k < 3; ++k) {
                    const double lo = dec_f64(a.lo[k]);
                    const double hi = dec_f64(a.hi[k]);
                    g.origin[k] = lo;
                    const double q = floor((hi - lo) / e);
                    if (!(q < 2147483646.0)) { err |= ERR_CAPACITY; break; }
                    g.dims[k] = (int32_t)q + 1;
                    prod *= g.dims[k];
                    if (prod >= 2147483647ll) { err |= ERR_CAPACITY; break; }
                }
                if (!err) nb = prod;
            }
            if (err) { nb = 0; g.dims[0] = g.dims[1] = g.dims[2] = 0; }
            g.error = (int32_t)err;
            g.n_boxes = nb;
        }
        long long tot;
        const long long base = block_excl_scan<long long>(nb, s_wave, tot);
        if (s < B) {
            const long long gb = running + base;
            g.box_base = gb < 2147483647ll ? (int32_t)gb : 0;
            geom[s] = g;
            if (err) atomicOr(&s_err, err);
        }
        running += tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t err = s_err;
        if (running > max_boxes || running >= 2147483647ll) err |= ERR_CAPACITY;
        hdr->need_boxes = running;
        hdr->error = err;
        hdr->total_boxes = err ? 0 : running;
        hdr->n_agents = n;
        hdr->n_sims = (uint32_t)B;
        uint32_t ep = hdr->epoch + 1u;
        if (ep >= (1u << 30)) ep = 1u;
        hdr->epoch = ep;
        hdr->scan_ticket = 0u;
    }
}

// ------------------------------------------------------------------- count

template <int M, bool BATCHED>
__global__ __launch_bounds__(kBlock) void k_count(const typename Mode<M>::In* __restrict__ x,
                                                  const typename Mode<M>::In* __restrict__ y,
                                                  const typename Mode<M>::In* __restrict__ z,
                                                  int64_t n, const int64_t* __restrict__ off,
                                                  int32_t B, const SimGeom* __restrict__ geom,
                                                  const Header* __restrict__ hdr,
                                                  int32_t* __restrict__ box_id,
                                                  int32_t* __restrict__ slot, int32_t* count)
{
    using Real = typename Mode<M>::Real;
    if (hdr->error) return;
    const int64_t i0 = (int64_t)blockIdx.x * kBlock;
    const int64_t i = i0 + threadIdx.x;
    int s = 0;
    if (BATCHED) {
        __shared__ int s_range[2];
        if (threadIdx.x == 0) {
            const int64_t last = (i0 + kBlock < n ? i0 + kBlock : n) - 1;
            s_range[0] = find_sim(off, 0, B, i0);
            s_range[1] = find_sim(off, 0, B, last);
        }
        __syncthreads();
        if (i < n) s = find_sim(off, s_range[0], s_range[1] + 1, i);
    }
    if (i >= n) return;
    const SimGeom g = geom[s];
    const int ix = axis_index((double)(Real)x[i], g.origin[0], g.edge, g.dims[0]);
    const int iy = axis_index((double)(Real)y[i], g.origin[1], g.edge, g.dims[1]);
    const int iz = axis_index((double)(Real)z[i], g.origin[2], g.edge, g.dims[2]);
    const int key = g.box_base + ix + g.dims[0] * (iy + g.dims[1] * iz);
    box_id[i] = key;
    slot[i] = atomicAdd(&count[key], 1);
}

// -------------------------------------------------------------------- scan

// Tile status word: [63:62] status (1 aggregate, 2 inclusive prefix),
// [61:32] build epoch, [31:0] value.
constexpr unsigned long long ST_AGG = 1ull, ST_INC = 2ull;

__device__ __forceinline__ unsigned long long make_flag(unsigned long long st, uint32_t epoch,
                                                        uint32_t v)
{
    return (st << 62) | ((unsigned long long)(epoch & 0x3fffffffu) << 32) | v;
}

__global__ __launch_bounds__(kBlock) void k_scan(Header* hdr, int32_t* count,
                                                 int32_t* __restrict__ start,
                                                 unsigned long long* flags)
{
    __shared__ uint32_t s_tile;
    __shared__ int32_t s_wave[kBlock / kWave];
    __shared__ int32_t s_prefix;
    if (hdr->error) return;
    const int64_t total = hdr->total_boxes;
    const int64_t len = total + 1;   // start[total] = number of agents
    const int64_t ntiles = (len + kScanTile - 1) / kScanTile;
    if (threadIdx.x == 0) s_tile = atomicAdd(&hdr->scan_ticket, 1u);
    __syncthreads();
    const int64_t t = s_tile;
    if (t >= ntiles) return;
    const uint32_t epoch = hdr->epoch;

    const int64_t base = t * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t idx = base + k;
        int32_t c = 0;
        if (idx < total) { c = count[idx]; count[idx] = 0; }
        v[k] = c;
        sum += c;
    }
    int32_t agg;
    const int32_t tp = block_excl_scan<int32_t>(sum, s_wave, agg);

    if (threadIdx.x < kWave) {
        const int lane = threadIdx.x;
        int64_t prefix = 0;
        if (t == 0) {
            if (lane == 0)
                __hip_atomic_store(&flags[0], make_flag(ST_INC, epoch, (uint32_t)agg),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(&flags[t], make_flag(ST_AGG, epoch, (uint32_t)agg),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t p = t - 1;   // window [p-63, p], lane l looks at p - l
            while (true) {
                const int64_t idx = p - lane;
                unsigned long long f = 0;
                unsigned long long st = 0;
                if (idx < 0) {
                    st = ST_INC;   // before the first tile: prefix 0
                } else {
                    do {
                        f = __hip_atomic_load(&flags[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const uint32_t fe = (uint32_t)(f >> 32) & 0x3fffffffu;
                        st = (fe == (epoch & 0x3fffffffu)) ? (f >> 62) : 0ull;
                    } while (st == 0);
                }
                const int64_t val = (idx < 0) ? 0 : (int64_t)(uint32_t)(f & 0xffffffffu);
                const unsigned long long inc = __ballot(st == ST_INC);
                if (inc) {
                    const int first = __ffsll((long long)inc) - 1;   // nearest inclusive
                    prefix += wave_sum<int64_t>(lane <= first ? val : 0);
                    break;
                }
                prefix += wave_sum<int64_t>(val);
                p -= kWave;
            }
            if (lane == 0)
                __hip_atomic_store(&flags[t], make_flag(ST_INC, epoch, (uint32_t)(prefix + agg)),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) s_prefix = (int32_t)prefix;
    }
    __syncthreads();
    int32_t run = s_prefix + tp;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t idx = base + k;
        if (idx < len) start[idx] = run;
        run += v[k];
    }
}

// ----------------------------------------------------------------- scatter

__global__ __launch_bounds__(kBlock) void k_scatter(const Header* __restrict__ hdr, int64_t n,
                                                    const int32_t* __restrict__ box_id,
                                                    const int32_t* __restrict__ slot,
                                                    const int32_t* __restrict__ start,
                                                    int32_t* __restrict__ perm_tmp)
{
    if (hdr->error) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    perm_tmp[start[box_id[i]] + slot[i]] = (int32_t)i;
}

// -------------------------------------------------------------------- rank

template <int M>
__global__ __launch_bounds__(kBlock) void k_rank(const typename Mode<M>::In* __restrict__ x,
                                                 const typename Mode<M>::In* __restrict__ y,
                                                 const typename Mode<M>::In* __restrict__ z,
                                                 const typename Mode<M>::In* __restrict__ d,
                                                 int64_t n, const Header* __restrict__ hdr,
                                                 const int32_t* __restrict__ box_id,
                                                 const int32_t* __restrict__ start,
                                                 const int32_t* __restrict__ perm_tmp,
                                                 int32_t* __restrict__ perm,
                                                 typename Mode<M>::Pay* __restrict__ pay)
{
    using Real = typename Mode<M>::Real;
    if (hdr->error) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int b = box_id[i];
    const int s0 = start[b], s1 = start[b + 1];
    int r = 0;
    for (int k = s0; k < s1; ++k) r += (perm_tmp[k] < (int32_t)i) ? 1 : 0;
    const int f = s0 + r;
    perm[f] = (int32_t)i;
    typename Mode<M>::Pay q;
    q.x = (Real)x[i];
    q.y = (Real)y[i];
    q.z = (Real)z[i];
    q.w = (Real)0.5 * (Real)d[i];
    pay[f] = q;
}

template <int M>
hipError_t grid_build_mode(const Layout& L, const Dev& D, const void* xv, const void* yv,
                           const void* zv, const void* dv, int64_t n, const int64_t* off,
                           int32_t B, double edge, const double* edges, hipStream_t s)
{
    using In = typename Mode<M>::In;
    const In* x = static_cast<const In*>(xv);
    const In* y = static_cast<const In*>(yv);
    const In* z = static_cast<const In*>(zv);
    const In* d = static_cast<const In*>(dv);
    const bool batched = off != nullptr;
    const int64_t* woff = nullptr;
    if (batched) {
        k_copy_offsets<<<(B + 1 + kBlock - 1) / kBlock, kBlock, 0, s>>>(off, D.off, B, n, D.acc);
        woff = D.off;
    }
    const unsigned nb_bounds = (unsigned)((n + kBoundsChunk - 1) / kBoundsChunk);
    if (batched)
        k_bounds<M, true><<<nb_bounds, kBlock, 0, s>>>(x, y, z, d, n, woff, B, D.acc);
    else
        k_bounds<M, false><<<nb_bounds, kBlock, 0, s>>>(x, y, z, d, n, nullptr, 1, D.acc);
    k_geometry<<<1, kBlock, 0, s>>>(D.hdr, D.acc, D.geom, woff, n, B, edge, edges, L.max_boxes);
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    if (batched)
        k_count<M, true><<<nb, kBlock, 0, s>>>(x, y, z, n, woff, B, D.geom, D.hdr, D.box_id,
                                                D.slot, D.count);
    else
        k_count<M, false><<<nb, kBlock, 0, s>>>(x, y, z, n, nullptr, 1, D.geom, D.hdr, D.box_id,
                                                 D.slot, D.count);
    k_scan<<<(unsigned)L.n_scan_tiles, kBlock, 0, s>>>(D.hdr, D.count, D.start, D.flags);
    k_scatter<<<nb, kBlock, 0, s>>>(D.hdr, n, D.box_id, D.slot, D.start, D.perm_tmp);
    k_rank<M><<<nb, kBlock, 0, s>>>(x, y, z, d, n, D.hdr, D.box_id, D.start, D.perm_tmp, D.perm,
                                    static_cast<typename Mode<M>::Pay*>(D.payload));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_init(const Layout& L, const Dev& D, hipStream_t s)
{
    k_init<<<512, kBlock, 0, s>>>(D.hdr, D.acc, L.max_sims, D.count, L.max_boxes + 1, D.flags,
                                  L.n_scan_tiles);
    return hipGetLastError();
}

hipError_t launch_grid_build(const Layout& L, const Dev& D, const void* x, const void* y,
                             const void* z, const void* d, int64_t n, const int64_t* off,
                             int32_t B, double edge, const double* edges, hipStream_t s)
{
    switch (L.dtype) {
    case MS_F32: return grid_build_mode<MS_F32>(L, D, x, y, z, d, n, off, B, edge, edges, s);
    case MS_F64: return grid_build_mode<MS_F64>(L, D, x, y, z, d, n, off, B, edge, edges, s);
    case MS_F32_POS64:
        return grid_build_mode<MS_F32_POS64>(L, D, x, y, z, d, n, off, B, edge, edges, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ms
