// Uniform-grid construction on the device (Section IV-A of the paper: a
// regular grid of boxes rebuilt every timestep; each box knows its agents).
//
// The paper keeps, per box, a count and the last agent added and links the
// agents of a box through a successor list.  Here the same information is a
// stable counting sort by box index held in the workspace: box start offsets,
// the box-sorted order perm (ascending box, then ascending input index) and a
// sorted copy of (x, y, z, d/2) for the force gather.
//
// Random-address global atomics and random scatters are the expensive
// operations on this GPU, so the sort is two-level and keeps the random work
// in LDS:
//   k_bounds      per (block, simulation) min/max of x, y, z and max diameter
//   k_geometry    one wave per simulation reduces its partials: edge (caller's
//                 or largest diameter), origin (minimum), dims
//                 (floor((max - min)/edge) + 1), box count, error bits
//   k_boxbase     global box range of every simulation, bucket size, error word
//   k_hist        box index per agent (FP64 binning) and a per-block LDS
//                 histogram over buckets (2^SB consecutive boxes)
//   k_rowscan     per bucket: exclusive scan over blocks of its counts and
//                 the bucket's total (the partition and the bucket sort
//                 recompute the bucket starts from the totals)
//   k_partition   agents moved into their bucket's range (slot from an LDS
//                 counter), carrying box index, input index and (x, y, z, d/2)
//   k_bucketsort  one block per bucket: LDS counting sort by box, box starts,
//                 then the stable rank of every agent among its box mates by
//                 input index, which fixes the canonical order exactly
#include "launch.hpp"

namespace ms {
namespace {

// ----------------------------------------------------------------- helpers

template <int NT, typename T>
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
    for (int w = 0; w < NT / kWave; ++w) {
        T t = s_wave[w];
        if (w < wid) wp += t;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return wp + x - v;
}

// Ranking into LDS counters with one atomic per run of equal keys among
// consecutive lanes: on box-sorted input whole wavefronts fall on one
// bucket, and a wavefront's atomics on one address are applied lane by lane.
// Every lane of the wavefront must call it.  Each lane with key >= 0 adds one
// to ctr[key] and gets its slot: the counter's value before its run plus the
// lane's place in the run, so the slots taken from one counter are distinct,
// as with one atomicAdd per lane (their order among lanes is not the same,
// and nothing here depends on it); a lane with key < 0 adds nothing.
// Measured in the tile partition (2M agents on the sorted state: 19.3 ->
// 14.6 us; 1% slower on random input); the histogram and the bucket sort,
// whose atomics were measured no faster with it, keep one atomic per lane.
__device__ __forceinline__ int wave_rank(int32_t* ctr, int key)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int prev = __shfl_up(key, 1);
    const bool head = lane == 0 || prev != key || key < 0;
    const uint64_t heads = __ballot(head);
    const uint64_t above = lane == kWave - 1 ? 0ull : (~0ull << (lane + 1));
    const uint64_t nxt = heads & above;
    const int end = nxt ? __builtin_ctzll(nxt) : kWave;
    int base = 0;
    if (head && key >= 0) base = atomicAdd(&ctr[key], end - lane);
    // the run's head: the highest head at or below this lane (lane 0 is one)
    const uint64_t upto = heads & (lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1));
    const int h = 63 - __builtin_clzll(upto);
    return __shfl(base, h) + (lane - h);
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}

// ------------------------------------------------------------------- init

__global__ void k_init(Header* hdr)
{
    if (threadIdx.x < sizeof(Header) / 4) reinterpret_cast<uint32_t*>(hdr)[threadIdx.x] = 0u;
}

__global__ void k_error_copy(const Header* __restrict__ hdr, int32_t* __restrict__ out)
{
    if (threadIdx.x == 0) out[0] = (int32_t)hdr->error;
}

// ------------------------------------------------------------- offsets copy

// Copies the caller's simulation offsets into the workspace and checks that
// they partition [0, n).
__global__ void k_copy_offsets(const int64_t* __restrict__ in, int64_t* out, int32_t B, int64_t n,
                               Header* hdr)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > B) return;
    const int64_t v = in[s];
    out[s] = v;
    bool bad = (v < 0) || (v > n) || (s == 0 && v != 0) || (s == B && v != n);
    if (s < B && in[s + 1] < v) bad = true;
    if (bad) atomicOr(&hdr->off_err, ERR_OFFSETS);
}

// ------------------------------------------------------------------ bounds

// Min/max over one whole chunk of a single simulation with 16-byte loads
// (all of a thread's loads issued before any is used), in the binning
// precision Real (exact: min and max only select), flags as k_bounds sets them.
template <int M>
__device__ __forceinline__ void bounds_chunk_vec(const typename Mode<M>::In* __restrict__ x,
                                                 const typename Mode<M>::In* __restrict__ y,
                                                 const typename Mode<M>::In* __restrict__ z,
                                                 const typename Mode<M>::In* __restrict__ d,
                                                 int64_t c0, double (&lo)[3], double (&hi)[3],
                                                 double& dm, uint32_t& fl)
{
    using In = typename Mode<M>::In;
    using Real = typename Mode<M>::Real;
    constexpr int V = 16 / (int)sizeof(In);            // agents per 16-byte load
    constexpr int U = kBoundsChunk / (kBlock * V);     // loads per thread and array
    static_assert(U * kBlock * V == kBoundsChunk, "whole loads per chunk");
    struct alignas(16) Vec { In v[V]; };
    const Vec* vx = reinterpret_cast<const Vec*>(x + c0);
    const Vec* vy = reinterpret_cast<const Vec*>(y + c0);
    const Vec* vz = reinterpret_cast<const Vec*>(z + c0);
    const Vec* vd = reinterpret_cast<const Vec*>(d + c0);
    Vec a[U], b[U], c[U], e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = u * kBlock + threadIdx.x;
        a[u] = vx[j]; b[u] = vy[j]; c[u] = vz[j]; e[u] = vd[j];
    }
    Real l[3] = {(Real)INFINITY, (Real)INFINITY, (Real)INFINITY};
    Real h[3] = {-(Real)INFINITY, -(Real)INFINITY, -(Real)INFINITY};
    Real m = -(Real)INFINITY;
    bool bad = false, neg = false;
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int t = 0; t < V; ++t) {
            const Real p[3] = {(Real)a[u].v[t], (Real)b[u].v[t], (Real)c[u].v[t]};
            const Real di = (Real)e[u].v[t];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                bad |= !isfinite(p[k]);
                l[k] = fmin(l[k], p[k]);
                h[k] = fmax(h[k], p[k]);
            }
            bad |= !isfinite(di);
            neg |= di < (Real)0;
            m = fmax(m, di);
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) { lo[k] = (double)l[k]; hi[k] = (double)h[k]; }
    dm = (double)m;
    fl = (bad ? (uint32_t)ERR_NONFINITE : 0u) | (neg ? (uint32_t)ERR_NEGDIAM : 0u);
}

// vec (single simulation only): the four input arrays are 16-byte aligned, so
// every whole chunk is read with bounds_chunk_vec.
template <int M, bool BATCHED>
__global__ __launch_bounds__(kBlock) void k_bounds(const typename Mode<M>::In* __restrict__ x,
                                                   const typename Mode<M>::In* __restrict__ y,
                                                   const typename Mode<M>::In* __restrict__ z,
                                                   const typename Mode<M>::In* __restrict__ d,
                                                   int64_t n, const int64_t* __restrict__ off,
                                                   int32_t B, BoundsPart* __restrict__ part,
                                                   bool vec)
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
        if (!BATCHED && vec && a1 - a0 == kBoundsChunk)   // block-uniform
            bounds_chunk_vec<M>(x, y, z, d, a0, lo, hi, dm, fl);
        else
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
            BoundsPart r;
            for (int k = 0; k < 3; ++k) { r.lo[k] = lo[k]; r.hi[k] = hi[k]; }
            r.dmax = dm;
            r.flags = fl;
            r.pad = 0;
            part[blockIdx.x + s] = r;   // (block, sim) pairs are unique at block + sim
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- geometry

// Geometry (Section IV-A: a uniform grid of boxes of edge e over the
// simulation's bounding box) from the reduced bounds: e = the caller's edge,
// or the largest diameter when it is <= 0; origin = the lower corner;
// dims = floor(extent / e) + 1 per axis.  nonempty: the simulation holds
// agents (an empty one gets no boxes).
__device__ SimGeom geometry_from(const double (&lo)[3], const double (&hi)[3], double dm,
                                 uint32_t fl, bool nonempty, double e)
{
    SimGeom g{};
    uint32_t err = fl;
    if (!isfinite(e)) err |= ERR_EDGE;
    else if (e <= 0.0) e = dm;
    g.edge = e;
    long long nb = 0;
    if (nonempty && err == 0) {
        if (!(e > 0.0) || e < dm) err |= ERR_EDGE;
    }
    if (nonempty && err == 0) {
        long long prod = 1;
        for (int k = 0; k < 3; ++k) {
            g.origin[k] = lo[k];
            const double q = floor((hi[k] - lo[k]) / e);
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
    return g;
}

// Geometry of the simulation holding agents [a0, a1) from its bounds partials
// (part[c + sh] for the chunks c it overlaps); a whole wave calls it and every
// lane gets the result.
__device__ SimGeom geometry_of(const BoundsPart* __restrict__ part, int64_t a0, int64_t a1, int sh,
                               double e)
{
    const int lane = threadIdx.x & (kWave - 1);
    double lo[3] = {INFINITY, INFINITY, INFINITY};
    double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double dm = -INFINITY;
    uint32_t fl = 0;
    if (a1 > a0) {
        const int64_t cl = a0 / kBoundsChunk, ch = (a1 - 1) / kBoundsChunk;
        for (int64_t c = cl + lane; c <= ch; c += kWave) {
            const BoundsPart& p = part[c + sh];
            for (int k = 0; k < 3; ++k) { lo[k] = fmin(lo[k], p.lo[k]); hi[k] = fmax(hi[k], p.hi[k]); }
            dm = fmax(dm, p.dmax);
            fl |= p.flags;
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) { lo[k] = wave_min(lo[k]); hi[k] = wave_max(hi[k]); }
    dm = wave_max(dm);
    fl = wave_or(fl);
    return geometry_from(lo, hi, dm, fl, a1 > a0, e);
}

// Batched builds: one wave per simulation (16 per block).
__global__ __launch_bounds__(1024) void k_geometry(const BoundsPart* __restrict__ part,
                                                   SimGeom* __restrict__ geom,
                                                   const int64_t* __restrict__ off, int64_t n,
                                                   int32_t B, double edge,
                                                   const double* __restrict__ edges)
{
    const int s = blockIdx.x * (1024 / kWave) + threadIdx.x / kWave;
    if (s >= B) return;   // wave-uniform
    const SimGeom g = geometry_of(part, off ? off[s] : 0, off ? off[s + 1] : n, off ? s : 0,
                                  edges ? edges[s] : edge);
    if ((threadIdx.x & (kWave - 1)) == 0) geom[s] = g;
}

// Bucket shift (buckets of 2^sb boxes holding about kBucketAgents agents on
// average, and no more buckets than the workspace holds) and count.
__device__ __forceinline__ void bucket_shape(long long boxes, int64_t n, int64_t nb_cap, int& sb,
                                             long long& nbk)
{
    sb = kSBMin;
    while (sb < kSBMax && (1ll << (sb + 1)) * n <= (long long)kBucketAgents * boxes) ++sb;
    while (sb < kSBMax && ((boxes + (1ll << sb) - 1) >> sb) > nb_cap) ++sb;
    nbk = (boxes + (1ll << sb) - 1) >> sb;
}

// Batched builds, one block: box base of every simulation, total boxes,
// bucket shift and count, the error word of the build, and start[total] = n.
__global__ __launch_bounds__(1024) void k_boxbase(Header* hdr, SimGeom* geom, int32_t B, int64_t n,
                                                  int64_t max_boxes, int64_t nb_cap,
                                                  int32_t* __restrict__ start)
{
    __shared__ long long s_wave[1024 / kWave];
    __shared__ uint32_t s_err;
    if (threadIdx.x == 0) s_err = 0;
    __syncthreads();
    long long running = 0;
    for (int c = 0; c < B; c += 1024) {
        const int s = c + threadIdx.x;
        long long nb = 0;
        if (s < B) {
            nb = geom[s].n_boxes;
            if (geom[s].error) atomicOr(&s_err, (uint32_t)geom[s].error);
        }
        long long tot;
        const long long base = block_excl_scan<1024, long long>(nb, s_wave, tot);
        if (s < B) {
            const long long gb = running + base;
            geom[s].box_base = gb < 2147483647ll ? (int32_t)gb : 0;
        }
        running += tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t err = s_err | hdr->off_err;
        hdr->off_err = 0u;
        if (running > max_boxes || running >= 2147483647ll) err |= ERR_CAPACITY;
        int sb;
        long long nbk;
        bucket_shape(running, n, nb_cap, sb, nbk);
        if (nbk > nb_cap) err |= ERR_CAPACITY;
        hdr->need_boxes = running;
        hdr->error = err;
        hdr->total_boxes = err ? 0 : running;
        hdr->n_agents = n;
        hdr->n_sims = (uint32_t)B;
        hdr->sb = sb;
        hdr->nb = err ? 0 : (int32_t)nbk;
        hdr->build_gen = hdr->build_gen + 1u;
        if (!err) start[running] = (int32_t)n;
    }
}

// ------------------------------------------------------- bucket histogram

// Row order of a single simulation's boxes (box_row): row-major, or, for
// `order` MS_BOX_ORDER_TILES or when MS_BOX_ORDER_AUTO finds many agents per
// z-plane, 16 x 16 tiles of rows.  An agent reads three z-planes of slots;
// row-major numbering puts its z-neighbour rows a whole plane of slots away,
// and once three planes outgrow an XCD's share of the L2 those rows are
// fetched again from HBM for every plane.  Inside a tile they are 16 rows
// away.  Auto keeps row-major when the tiles' padding would add more than a
// quarter to the box count or not fit the workspace.  Sets g.tile_shift and,
// for tiles, the padded g.n_boxes.
__device__ void choose_rows(SimGeom& g, int64_t n, int64_t max_boxes, int order)
{
    g.tile_shift = 0;
    if (g.error || g.n_boxes <= 0 || order == MS_BOX_ORDER_ROWS) return;
    const bool autom = order != MS_BOX_ORDER_TILES;
    if (autom && n < kTilePlaneAgents * (int64_t)g.dims[2]) return;
    const int s = kRowTileShift, m = (1 << s) - 1;
    const long long nty = (g.dims[1] + (long long)m) >> s, lz = g.dims[2] - 1;
    // 1 + box_row of the last tile's last row, in 64 bits
    const long long rows = ((((lz >> s) * nty + nty - 1) << (2 * s)) | ((lz & m) << s)) + m + 1;
    const long long nb = (long long)g.dims[0] * rows;
    if (autom && (4 * nb > 5 * g.n_boxes || nb > max_boxes)) return;
    g.tile_shift = s;
    g.n_boxes = nb;
}

// Single simulation: the build's shape from its geometry g (row order,
// error word, bucket shift and count) into s_geo / s_shape (shift, bucket
// count, error); with `write` also the geometry, the build header and
// start[boxes] = n.
__device__ void publish_single(SimGeom g, int64_t n, int64_t max_boxes, int64_t nb_cap, int order,
                               bool write, SimGeom* __restrict__ geom, Header* __restrict__ hdr,
                               int32_t* __restrict__ start, SimGeom& s_geo, int (&s_shape)[3])
{
    choose_rows(g, n, max_boxes, order);
    uint32_t err = (uint32_t)g.error;
    const long long boxes = g.n_boxes;
    if (boxes > max_boxes || boxes >= 2147483647ll) err |= ERR_CAPACITY;
    int shift;
    long long nb;
    bucket_shape(boxes, n, nb_cap, shift, nb);
    if (nb > nb_cap) err |= ERR_CAPACITY;
    g.box_base = 0;
    s_geo = g;
    s_shape[0] = shift;
    s_shape[1] = err ? 0 : (int)nb;
    s_shape[2] = (int)err;
    if (write) {
        geom[0] = g;
        hdr->off_err = 0u;
        hdr->need_boxes = boxes;
        hdr->error = err;
        hdr->total_boxes = err ? 0 : boxes;
        hdr->n_agents = n;
        hdr->n_sims = 1u;
        hdr->sb = shift;
        hdr->nb = err ? 0 : (int32_t)nb;
        hdr->build_gen = hdr->build_gen + 1u;
        hdr->nchunk = 0u;
        if (!err) start[boxes] = (int32_t)n;
    }
}

// Bounds partials above which a single-simulation build reduces them in a
// launch of its own (k_geometry1) rather than in every histogram block.
constexpr int kGeomSplit = 1024;
// Blocks of the chunk sort of such builds (three per CU).
constexpr int kSortChunkBlocks = 768;

// Zero the (bucket x tile) count matrix of a large single build, whose
// histogram then writes only nonzero counts.  Sized by the bucket count the
// geometry reduction published.
__global__ __launch_bounds__(kBlock) void k_clear_hist(const Header* __restrict__ hdr,
                                                       int32_t* __restrict__ hist, int32_t nblk)
{
    if (hdr->error) return;
    const int64_t total = (int64_t)hdr->nb * nblk;
    const int64_t n4 = total / 4;
    int4* h4 = reinterpret_cast<int4*>(hist);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride)
        h4[i] = make_int4(0, 0, 0, 0);
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += stride)
        hist[i] = 0;
}

static_assert(kTileThreads == 1024, "block_bounds runs on blocks of 1,024 threads");

// Bounds of a single simulation from its nc partials, reduced by a whole
// block of 1,024 threads (U partials per thread loaded before any is
// reduced); valid in thread 0.  Every thread of the block must call it.
struct BlockBounds {
    double red[7][1024 / kWave];
    uint32_t fl[1024 / kWave];
};

template <int U>
__device__ void block_bounds(const BoundsPart* __restrict__ part, int64_t nc, BlockBounds& sm,
                             double (&lo)[3], double (&hi)[3], double& dm, uint32_t& fl)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    dm = -INFINITY;
    fl = 0;
    for (int64_t c0 = threadIdx.x; c0 < nc; c0 += 1024 * U) {
        BoundsPart p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t c = c0 + 1024 * u;
            if (c < nc) {
                p[u] = part[c];
            } else {
                for (int k = 0; k < 3; ++k) { p[u].lo[k] = INFINITY; p[u].hi[k] = -INFINITY; }
                p[u].dmax = -INFINITY;
                p[u].flags = 0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            for (int k = 0; k < 3; ++k) {
                lo[k] = fmin(lo[k], p[u].lo[k]);
                hi[k] = fmax(hi[k], p[u].hi[k]);
            }
            dm = fmax(dm, p[u].dmax);
            fl |= p[u].flags;
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) { lo[k] = wave_min(lo[k]); hi[k] = wave_max(hi[k]); }
    dm = wave_max(dm);
    fl = wave_or(fl);
    if (lane == 0) {
        for (int k = 0; k < 3; ++k) { sm.red[k][wid] = lo[k]; sm.red[3 + k][wid] = hi[k]; }
        sm.red[6][wid] = dm;
        sm.fl[wid] = fl;
    }
    __syncthreads();
    if (wid == 0) {
        // the 16 wave results, one per lane, reduced by wave 0
        const bool on = lane < 1024 / kWave;
        for (int k = 0; k < 3; ++k) {
            lo[k] = wave_min(on ? sm.red[k][lane] : INFINITY);
            hi[k] = wave_max(on ? sm.red[3 + k][lane] : -INFINITY);
        }
        dm = wave_max(on ? sm.red[6][lane] : -INFINITY);
        fl = wave_or(on ? sm.fl[lane] : 0u);
    }
}

// Single simulation with many bounds partials (more than kGeomSplit): one
// block of 1,024 threads reduces them all and publishes geometry and header
// once, instead of every histogram block reducing them.
__global__ __launch_bounds__(1024) void k_geometry1(const BoundsPart* __restrict__ part,
                                                    int64_t n, double edge, int64_t max_boxes,
                                                    int64_t nb_cap, int order,
                                                    SimGeom* __restrict__ geom,
                                                    Header* __restrict__ hdr,
                                                    int32_t* __restrict__ start)
{
    __shared__ BlockBounds s_bb;
    __shared__ SimGeom s_geo;
    __shared__ int s_shape[3];
    double lo[3], hi[3], dm;
    uint32_t fl;
    block_bounds<4>(part, (n + kBoundsChunk - 1) / kBoundsChunk, s_bb, lo, hi, dm, fl);
    if (threadIdx.x == 0) {
        const SimGeom g = geometry_from(lo, hi, dm, fl, n > 0, edge);
        publish_single(g, n, max_boxes, nb_cap, order, true, geom, hdr, start, s_geo, s_shape);
    }
}

template <int M, bool BATCHED, bool PRE>
__global__ __launch_bounds__(kTileThreads) void k_hist(const typename Mode<M>::In* __restrict__ x,
                                                 const typename Mode<M>::In* __restrict__ y,
                                                 const typename Mode<M>::In* __restrict__ z,
                                                 int64_t n, const int64_t* __restrict__ off,
                                                 int32_t B, SimGeom* __restrict__ geom,
                                                 Header* __restrict__ hdr,
                                                 int32_t* __restrict__ box_id,
                                                 uint8_t* __restrict__ quarter,
                                                 int32_t* __restrict__ hist,
                                                 const BoundsPart* __restrict__ part, double edge,
                                                 int64_t max_boxes, int64_t nb_cap, int order,
                                                 int32_t* __restrict__ start)
{
    using Real = typename Mode<M>::Real;
    using In = typename Mode<M>::In;
    __shared__ int32_t h[kBucketsMax];
    __shared__ int s_range[2];
    __shared__ SimGeom s_geo;
    __shared__ int s_shape[3];   // sb, nb, error
    const unsigned tile = xcd_block();
    const int64_t c0 = (int64_t)tile * kTileA;
    const int64_t c1 = (c0 + kTileA < n) ? c0 + kTileA : n;
    int sb, nbk;
    if (BATCHED) {
        if (hdr->error) return;
        sb = hdr->sb;
        nbk = hdr->nb;
    } else {
        // One simulation: up to kGeomSplit bounds partials every block
        // reduces them itself (a launch of its own costs more at that size)
        // and block 0 publishes the geometry and the build header for the
        // later passes; above it k_geometry1 has done both.
        if (PRE) {
            // geometry and header published by k_geometry1
            if (threadIdx.x == 0) {
                s_geo = geom[0];
                s_shape[0] = hdr->sb;
                s_shape[1] = hdr->nb;
                s_shape[2] = (int)hdr->error;
            }
        } else if (threadIdx.x < kWave) {
            const SimGeom g = geometry_of(part, 0, n, 0, edge);
            if (threadIdx.x == 0)
                publish_single(g, n, max_boxes, nb_cap, order, blockIdx.x == 0, geom, hdr, start,
                               s_geo, s_shape);
        }
        __syncthreads();
        if (s_shape[2]) return;   // block-uniform
        sb = s_shape[0];
        nbk = s_shape[1];
    }
    for (int b = threadIdx.x; b < nbk; b += kTileThreads) h[b] = 0;
    if (BATCHED && threadIdx.x == 0) {
        s_range[0] = find_sim(off, 0, B, c0);
        s_range[1] = find_sim(off, 0, B, c1 - 1);
    }
    __syncthreads();
    auto bin = [&](int64_t i, const SimGeom& g, In xi, In yi, In zi) {
        const double px = (double)(Real)xi;
        const int ix = axis_index(px, g.origin[0], g.edge, g.dims[0]);
        const int iy = axis_index((double)(Real)yi, g.origin[1], g.edge, g.dims[1]);
        const int iz = axis_index((double)(Real)zi, g.origin[2], g.edge, g.dims[2]);
        const int key = g.box_base + ix + g.dims[0] * box_row(iy, iz, g.dims[1], g.tile_shift);
        box_id[i] = key;
        quarter[i] = (uint8_t)box_quarter(px, g.origin[0], 4.0 / g.edge, g.edge, ix);
        // box-sorted input puts a whole wavefront in one bucket: one LDS
        // atomic then counts it, instead of 64 on the same address
        const int bk = key >> sb;
        const int bf = __builtin_amdgcn_readfirstlane(bk);
        const uint64_t act = __ballot(1);
        if (__ballot(bk == bf) == act) {
            if ((int)(threadIdx.x & (kWave - 1)) == (int)__ffsll((unsigned long long)act) - 1)
                atomicAdd(&h[bf], (int)__popcll(act));
        } else {
            atomicAdd(&h[bk], 1);
        }
    };
    for (int64_t i = c0 + threadIdx.x; i < c1; i += kTileThreads) {
        const int s = BATCHED ? find_sim(off, s_range[0], s_range[1] + 1, i) : 0;
        bin(i, BATCHED ? geom[s] : s_geo, x[i], y[i], z[i]);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbk; b += kTileThreads)
        // large single builds (PRE) cleared the matrix beforehand and write
        // only the buckets this tile touches: a tile of box-sorted input
        // falls into a few buckets, and each 4-byte store of a zero column
        // entry costs a whole memory sector
        if (!PRE || h[b] != 0) hist[(int64_t)b * gridDim.x + tile] = h[b];
}

// One block per bucket: exclusive scan along its row of per-block counts.
__global__ __launch_bounds__(kBlock) void k_rowscan(const Header* __restrict__ hdr,
                                                    int32_t* __restrict__ hist, int32_t nblk,
                                                    int32_t* __restrict__ btot)
{
    __shared__ int32_t s_wave[kBlock / kWave];
    if (hdr->error) return;
    const int b = blockIdx.x;
    if (b >= hdr->nb) return;
    int32_t* row = hist + (int64_t)b * nblk;
    constexpr int IT = 4;
    int32_t running = 0;
    for (int c = 0; c < nblk; c += kBlock * IT) {
        int32_t v[IT];
        int32_t sum = 0;
        const int base = c + threadIdx.x * IT;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            v[k] = (base + k < nblk) ? row[base + k] : 0;
            sum += v[k];
        }
        int32_t tot;
        int32_t ex = block_excl_scan<kBlock, int32_t>(sum, s_wave, tot) + running;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            if (base + k < nblk) row[base + k] = ex;
            ex += v[k];
        }
        running += tot;
    }
    if (threadIdx.x == 0) btot[b] = running;
}

// Where the bucket sort takes an agent's sorted payload (x, y, z, d/2) from:
// the partition's copy, or (GATHER) the inputs at its input index.  Builds
// whose inputs are nearly box-sorted (the workspace's sorted_input switch:
// the state a sorted-state step or a reorder wrote) take GATHER: the inputs
// of one bucket are then nearly contiguous, and the partition skips reading
// and writing the payload.  It is only a question of speed: both give the
// same build for any input.
template <int M, bool GATHER>
struct PaySrc {
    using In = typename Mode<M>::In;
    using Real = typename Mode<M>::Real;
    using Pay = typename Mode<M>::Pay;
    const Pay* pay2;
    const In *x, *y, *z, *d;
    __device__ __forceinline__ Pay get(int64_t pos, int64_t id) const
    {
        if constexpr (!GATHER) return pay2[pos];
        Pay q;
        q.x = (Real)x[id];
        q.y = (Real)y[id];
        q.z = (Real)z[id];
        q.w = (Real)0.5 * (Real)d[id];
        return q;
    }
};

// ---------------------------------------------------------------- partition

// Each block orders its tile by bucket in LDS, then writes every bucket's run
// contiguously (consecutive lanes -> consecutive addresses), reading the
// agents' inputs inside the tile.
template <int M, bool GATHER>
__global__ __launch_bounds__(kTileThreads) void k_partition(const typename Mode<M>::In* __restrict__ x,
                                                      const typename Mode<M>::In* __restrict__ y,
                                                      const typename Mode<M>::In* __restrict__ z,
                                                      const typename Mode<M>::In* __restrict__ d,
                                                      int64_t n, const Header* __restrict__ hdr,
                                                      const int32_t* __restrict__ box_id,
                                                      const uint8_t* __restrict__ quarter,
                                                      const int32_t* __restrict__ hist,
                                                      const int32_t* __restrict__ btot,
                                                      int32_t* __restrict__ key2,
                                                      int32_t* __restrict__ idx2,
                                                      typename Mode<M>::Pay* __restrict__ pay2)
{
    using Real = typename Mode<M>::Real;
    constexpr int IT = kTileA / kTileThreads;
    __shared__ int32_t cnt[kBucketsMax];     // tile counts, then tile-local bucket starts
    __shared__ int32_t gcur[kBucketsMax];    // global start of this tile's run per bucket
    __shared__ uint16_t order[kTileA];       // tile-local index in bucket order
    __shared__ int32_t s_wave[kTileThreads / kWave];
    if (hdr->error) return;
    const int sb = hdr->sb, nbk = hdr->nb;
    constexpr bool gat = GATHER;
    for (int b = threadIdx.x; b < nbk; b += kTileThreads) cnt[b] = 0;
    __syncthreads();
    const unsigned tile = xcd_block();   // consecutive tiles on one XCD
    const int64_t c0 = (int64_t)tile * kTileA;
    const int tn = (int)((c0 + kTileA < n) ? kTileA : n - c0);
    int bk[IT], rk[IT];
#pragma unroll
    for (int t = 0; t < IT; ++t) {
        const int e = threadIdx.x + t * kTileThreads;
        bk[t] = e < tn ? box_id[c0 + e] >> sb : -1;
    }
#pragma unroll
    for (int t = 0; t < IT; ++t) rk[t] = wave_rank(cnt, bk[t]);
    __syncthreads();
    // exclusive scan of the tile counts over buckets; global run starts
    const int per = (nbk + kTileThreads - 1) / kTileThreads;
    const int b0 = threadIdx.x * per;
    // the tile's counts and the bucket totals are scanned together: the
    // bucket starts (exclusive scan of the totals) are recomputed by every
    // block, which is cheaper than a launch of their own
    int32_t sum = 0, sumb = 0;
    for (int b = b0; b < b0 + per && b < nbk; ++b) {
        sum += cnt[b];
        sumb += btot[b];
    }
    int32_t tot, totb;
    int32_t run = block_excl_scan<kTileThreads, int32_t>(sum, s_wave, tot);
    int32_t runb = block_excl_scan<kTileThreads, int32_t>(sumb, s_wave, totb);
    for (int b = b0; b < b0 + per && b < nbk; ++b) {
        const int32_t v = cnt[b];
        cnt[b] = run;
        gcur[b] = runb + hist[(int64_t)b * gridDim.x + tile] - run;
        run += v;
        runb += btot[b];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < IT; ++t) {
        const int e = threadIdx.x + t * kTileThreads;
        if (e < tn) order[cnt[bk[t]] + rk[t]] = (uint16_t)e;
    }
    __syncthreads();
    // gather inside the tile (all loads of a group issued before any store);
    // in gather mode the bucket sort reads the payload from the inputs itself
    constexpr int G = 4;
    for (int p0 = threadIdx.x; p0 < tn; p0 += G * kTileThreads) {
        int64_t i[G];
        int key[G], qx[G];
        typename Mode<M>::Pay q[G];
#pragma unroll
        for (int t = 0; t < G; ++t) {
            const int p = p0 + t * kTileThreads;
            i[t] = c0 + order[p < tn ? p : tn - 1];
        }
#pragma unroll
        for (int t = 0; t < G; ++t) {
            key[t] = box_id[i[t]];
            qx[t] = quarter[i[t]];
            if (!gat) {
                q[t].x = (Real)x[i[t]];
                q[t].y = (Real)y[i[t]];
                q[t].z = (Real)z[i[t]];
                q[t].w = (Real)0.5 * (Real)d[i[t]];
            }
        }
#pragma unroll
        for (int t = 0; t < G; ++t) {
            const int p = p0 + t * kTileThreads;
            if (p < tn) {
                const int pos = gcur[key[t] >> sb] + p;
                key2[pos] = ((key[t] & ((1 << sb) - 1)) << 2) | qx[t];
                idx2[pos] = (int32_t)i[t];
                if (!gat) pay2[pos] = q[t];
            }
        }
    }
}

// FP32 payloads: the same partition with the permutation done in LDS.  Each
// thread loads its own agents (coalesced), they are placed in bucket order in
// LDS (key, tile position + quarter, payload), and each bucket run is then
// written from LDS in order.  One block per CU (the tile needs ~120 KB).
template <int M, bool GATHER>
__global__ __launch_bounds__(kTileThreads) void k_partition_lds(const typename Mode<M>::In* __restrict__ x,
                                                                const typename Mode<M>::In* __restrict__ y,
                                                                const typename Mode<M>::In* __restrict__ z,
                                                                const typename Mode<M>::In* __restrict__ d,
                                                                int64_t n, const Header* __restrict__ hdr,
                                                                const int32_t* __restrict__ box_id,
                                                                const uint8_t* __restrict__ quarter,
                                                                const int32_t* __restrict__ hist,
                                                                const int32_t* __restrict__ btot,
                                                                int32_t* __restrict__ key2,
                                                                int32_t* __restrict__ idx2,
                                                                F4* __restrict__ pay2)
{
    using Real = typename Mode<M>::Real;
    static_assert(sizeof(typename Mode<M>::Pay) == sizeof(F4), "FP32 payloads only");
    static_assert(kTileA <= 4096, "tile positions are 12-bit");
    constexpr int IT = kTileA / kTileThreads;
    // tile counts, then tile-local bucket starts, then (global start of this
    // tile's run - tile-local start) per bucket: one array, so that two
    // gather-mode blocks fit a CU's LDS
    __shared__ int32_t cnt[kBucketsMax];
    __shared__ int32_t s_key[kTileA];        // box index, bucket order
    __shared__ uint16_t s_eq[kTileA];        // tile position | quarter << 12, bucket order
    __shared__ F4 s_pay[kTileA];             // (x, y, z, d/2), bucket order
    __shared__ int32_t s_wave[kTileThreads / kWave];
    constexpr int PER = (kBucketsMax + kTileThreads - 1) / kTileThreads;   // buckets per thread
    if (hdr->error) return;
    const int sb = hdr->sb, nbk = hdr->nb;
    // in gather mode the bucket sort reads the payload from the inputs itself
    constexpr bool gat = GATHER;
    for (int b = threadIdx.x; b < nbk; b += kTileThreads) cnt[b] = 0;
    __syncthreads();
    const unsigned tile = xcd_block();   // consecutive tiles on one XCD
    const int64_t c0 = (int64_t)tile * kTileA;
    const int tn = (int)((c0 + kTileA < n) ? kTileA : n - c0);
    int key[IT], rk[IT], qx[IT];
    F4 q[IT];
#pragma unroll
    for (int t = 0; t < IT; ++t) {
        const int e = threadIdx.x + t * kTileThreads;
        key[t] = -1;
        if (e < tn) {
            const int64_t i = c0 + e;
            key[t] = box_id[i];
            qx[t] = quarter[i];
            if (!gat) {
                q[t].x = (Real)x[i];
                q[t].y = (Real)y[i];
                q[t].z = (Real)z[i];
                q[t].w = (Real)0.5 * (Real)d[i];
            }
        }
    }
#pragma unroll
    for (int t = 0; t < IT; ++t) rk[t] = wave_rank(cnt, key[t] >= 0 ? key[t] >> sb : -1);
    __syncthreads();
    // exclusive scan of the tile counts over buckets; global run starts
    const int per = (nbk + kTileThreads - 1) / kTileThreads;
    const int b0 = threadIdx.x * per;
    // the tile's counts and the bucket totals are scanned together: the
    // bucket starts (exclusive scan of the totals) are recomputed by every
    // block, which is cheaper than a launch of their own
    int32_t sum = 0, sumb = 0;
    for (int b = b0; b < b0 + per && b < nbk; ++b) {
        sum += cnt[b];
        sumb += btot[b];
    }
    int32_t tot, totb;
    int32_t run = block_excl_scan<kTileThreads, int32_t>(sum, s_wave, tot);
    int32_t runb = block_excl_scan<kTileThreads, int32_t>(sumb, s_wave, totb);
    int32_t gofs[PER];   // this thread's buckets: global run start - tile-local start
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int b = b0 + j;
        gofs[j] = 0;
        if (j < per && b < nbk) {
            const int32_t v = cnt[b];
            cnt[b] = run;
            gofs[j] = runb + hist[(int64_t)b * gridDim.x + tile] - run;
            run += v;
            runb += btot[b];
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < IT; ++t) {
        if (key[t] >= 0) {
            const int e = threadIdx.x + t * kTileThreads;
            const int pos = cnt[key[t] >> sb] + rk[t];
            s_key[pos] = key[t];
            s_eq[pos] = (uint16_t)(e | (qx[t] << 12));
            if (!gat) s_pay[pos] = q[t];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j)
        if (j < per && b0 + j < nbk) cnt[b0 + j] = gofs[j];
    __syncthreads();
    // bucket runs written in order: consecutive threads, consecutive addresses
    for (int p = threadIdx.x; p < tn; p += kTileThreads) {
        const int k = s_key[p];
        const int eq = s_eq[p];
        const int pos = cnt[k >> sb] + p;
        key2[pos] = ((k & ((1 << sb) - 1)) << 2) | (eq >> 12);
        idx2[pos] = (int32_t)(c0 + (eq & 0xfff));
        if (!gat) pay2[pos] = s_pay[p];
    }
}

// -------------------------------------------------------------- bucket sort

constexpr int kSortBoxes = 1 << kSBMax;
static_assert(kSortStage <= 4096 && kSortBoxes <= 4096,
              "the chunk sort packs a box and an arrival slot in 12 bits each");

// Quarter counts of one box member, packed as the split word's bytes 0..2
// (members in quarters below 1, 2, 3).
__device__ __forceinline__ uint32_t split_inc(int q)
{
    return (q < 1 ? 1u : 0u) | (q < 2 ? 0x100u : 0u) | (q < 3 ? 0x10000u : 0u);
}

// Split word of a box of cnt agents from its packed quarter counts.
__device__ __forceinline__ uint32_t split_word(uint32_t w, int cnt)
{
    return cnt > 255 ? kSplitNone : (w | ((uint32_t)cnt << 24));
}

// Quantised copy of each slot for the gather's candidate test (the test and
// why it never rejects a contact are in gather.hpp): x, y, z relative to the
// simulation's grid origin in units of e / kQuantScale rounded down, kept
// modulo 2^16, and the radius in the same units rounded up and negated, as
// ((x | y << 16), (z | -r << 16)).  The positions are the payload's (the
// values the force uses).  A batched build quantises each slot in its own
// simulation's frame (agents of different simulations never meet); the
// simulations of a bucket's boxes are found once per bucket.
struct SlotQ {
    uint2* p;
    const SimGeom* g;
    int slo, shi;   // simulations holding the bucket's first and last box
    __device__ SlotQ(uint2* payq, const SimGeom* geom, int s_lo, int s_hi)
        : p(payq), g(geom), slo(s_lo), shi(s_hi) {}
    __device__ static uint32_t q16(double v) { return (uint32_t)(int64_t)floor(v) & 0xffffu; }
    // gbox: global box of the slot's agent
    template <typename Pay>
    __device__ __forceinline__ void put(int slot, const Pay& q, int gbox) const
    {
        int lo = slo, hi = shi + 1;   // the last simulation with box_base <= gbox
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (g[mid].box_base <= gbox) lo = mid; else hi = mid;
        }
        const SimGeom& f = g[lo];
        const double sc = (double)kQuantScale / f.edge;
        const uint32_t xq = q16(((double)q.x - f.origin[0]) * sc);
        const uint32_t yq = q16(((double)q.y - f.origin[1]) * sc);
        const uint32_t zq = q16(((double)q.z - f.origin[2]) * sc);
        const int rq = (int)ceil((double)q.w * sc);
        p[slot] = make_uint2(xq | (yq << 16), zq | ((uint32_t)(-rq) << 16));
    }
};

// Simulation of global box gbox among sims [0, B): the last with box_base <= gbox.
__device__ __forceinline__ int sim_of_box(const SimGeom* __restrict__ g, int B, int gbox)
{
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (g[mid].box_base <= gbox) lo = mid; else hi = mid;
    }
    return lo;
}

// Buckets holding more agents than the LDS stage: after the box counts, box
// starts and the arrival-order placement (tmp[s0 + slot] = position of the
// slot's agent in the bucket input, c[k] = end of box k), the boxes are taken
// in consecutive chunks of at most kSortStage agents.  Each chunk's members
// are loaded into LDS once, ranked among their box mates by (quarter, input
// index) there, and written in slot order; a member's box is the one whose
// slot range holds its arrival slot.  A single box above kSortStage agents is
// ranked straight from global memory.
// The chunk that starts at box kb (first slot cs, relative to the bucket's
// start): boxes [kb, ke) ending at or before cs + kSortStage, or the single
// box kb if that alone is larger; ce: its end slot.  c[k]: end of box k.
__device__ __forceinline__ void chunk_end(const int32_t* c, int nbox, int kb, int cs, int& ke,
                                          int& ce)
{
    int lo = kb, hi = nbox;   // first box ending beyond the limit lies in [lo, hi]
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (c[mid] - cs > kSortStage) hi = mid; else lo = mid + 1;
    }
    ke = lo > kb ? lo : kb + 1;
    ce = c[ke - 1];
}

// Sort one chunk (boxes [kb, ke), slots [cs, ce) of the bucket starting at
// slot s0 and box b0): c[k] (k in [kb - 1, ke)) holds box ends relative to s0.
template <int M, bool GATHER>
__device__ void sort_chunk(int s0, int b0, int kb, int ke, int cs, int ce, const int32_t* c,
                           int32_t* mem, uint8_t* memq, int32_t* inv,
                           const int32_t* __restrict__ key2, const int32_t* __restrict__ idx2,
                           const PaySrc<M, GATHER>& src, const int32_t* __restrict__ tmp,
                           uint32_t* __restrict__ split, int32_t* __restrict__ perm,
                           typename Mode<M>::Pay* __restrict__ pay, const SlotQ& s32)
{
    const int cn = ce - cs;
    if (cn <= kSortStage) {
        // each thread's (at most U) members: all loads issued before any use
        constexpr int U = kSortStage / kSortThreads;
        static_assert(U * kSortThreads == kSortStage, "whole rounds per chunk");
        int pm[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = threadIdx.x + u * kSortThreads;
            pm[u] = j < cn ? tmp[s0 + cs + j] : 0;
        }
        int32_t id[U], kq[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            id[u] = idx2[s0 + pm[u]];
            kq[u] = key2[s0 + pm[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = threadIdx.x + u * kSortThreads;
            if (j < cn) {
                mem[j] = id[u];
                memq[j] = (uint8_t)(kq[u] & 3);
            }
        }
        __syncthreads();
        for (int j = threadIdx.x; j < cn; j += kSortThreads) {
            int k0 = kb, k1 = ke - 1;   // box of arrival slot cs + j: first with c[k] > cs + j
            while (k0 < k1) {
                const int mid = (k0 + k1) >> 1;
                if (c[mid] > cs + j) k1 = mid; else k0 = mid + 1;
            }
            const int k = k0, q = memq[j];
            const int32_t orig = mem[j];
            const int bs = (k > 0 ? c[k - 1] : 0) - cs, be = c[k] - cs;
            int r = 0;
            uint32_t w = 0;
            for (int m = bs; m < be; ++m) {
                const int qm = memq[m];
                r += (qm < q || (qm == q && mem[m] < orig)) ? 1 : 0;
                w += split_inc(qm);
            }
            if (r == 0)
                reinterpret_cast<uint2*>(split)[b0 + k] =
                    make_uint2((uint32_t)(s0 + cs + bs), split_word(w, be - bs));
            // final slot -> box within the chunk (bits 12..23), arrival slot
            inv[bs + r] = ((k - kb) << 12) | j;
        }
        __syncthreads();
        // FP64 inputs are written in two halves (fewer 8-byte values in
        // flight, as in the staged path).  The box and the input index come
        // from LDS; only the carry mode still reads the member's position.
        constexpr int HALVES = 2;
        constexpr int UH = U / HALVES;
#pragma unroll
        for (int hh = 0; hh < HALVES; ++hh) {
            int jj[UH], pw[UH], bx[UH];
#pragma unroll
            for (int u = 0; u < UH; ++u) {
                const int p = threadIdx.x + (hh * UH + u) * kSortThreads;
                const int v = p < cn ? inv[p] : 0;   // padding lanes use arrival slot 0
                jj[u] = v & 4095;
                bx[u] = b0 + kb + (v >> 12);
                pw[u] = 0;
                if constexpr (!GATHER) pw[u] = tmp[s0 + cs + jj[u]];
            }
            typename Mode<M>::Pay q[UH];
#pragma unroll
            for (int u = 0; u < UH; ++u) q[u] = src.get(s0 + pw[u], mem[jj[u]]);
#pragma unroll
            for (int u = 0; u < UH; ++u) {
                const int p = threadIdx.x + (hh * UH + u) * kSortThreads;
                if (p < cn) {
                    perm[s0 + cs + p] = mem[jj[u]];
                    pay[s0 + cs + p] = q[u];
                    s32.put(s0 + cs + p, q[u], bx[u]);
                }
            }
        }
        __syncthreads();
    } else {
        // one box (ke = kb + 1) larger than the stage
        const int k = kb;
        for (int j = threadIdx.x; j < cn; j += kSortThreads) {
            const int pe = tmp[s0 + cs + j];
            const int q = key2[s0 + pe] & 3;
            const int32_t orig = idx2[s0 + pe];
            int r = 0;
            for (int m = 0; m < cn; ++m) {
                const int pm = tmp[s0 + cs + m];
                const int qm = key2[s0 + pm] & 3;
                r += (qm < q || (qm == q && idx2[s0 + pm] < orig)) ? 1 : 0;
            }
            if (r == 0)
                reinterpret_cast<uint2*>(split)[b0 + k] = make_uint2((uint32_t)(s0 + cs), kSplitNone);
            perm[s0 + cs + r] = orig;
            const typename Mode<M>::Pay qv = src.get(s0 + pe, orig);
            pay[s0 + cs + r] = qv;
            s32.put(s0 + cs + r, qv, b0 + k);
        }
    }
}

template <int M, bool GATHER>
__device__ void sort_chunks(int s0, int nbox, int b0, const int32_t* c, int32_t* mem, uint8_t* memq,
                            int32_t* inv, const int32_t* __restrict__ key2,
                            const int32_t* __restrict__ idx2,
                            const PaySrc<M, GATHER>& src,
                            const int32_t* __restrict__ tmp, uint32_t* __restrict__ split,
                            int32_t* __restrict__ perm, typename Mode<M>::Pay* __restrict__ pay,
                            const SlotQ& s32)
{
    int kb = 0, cs = 0;   // first box and first slot of the chunk (block-uniform)
    while (kb < nbox) {
        int ke, ce;
        chunk_end(c, nbox, kb, cs, ke, ce);
        sort_chunk<M, GATHER>(s0, b0, kb, ke, cs, ce, c, mem, memq, inv, key2, idx2, src, tmp,
                              split, perm, pay, s32);
        kb = ke;
        cs = ce;
    }
}

// Six wavefronts per SIMD (at most 80 VGPRs; the slot-order writes go out in
// two halves so that no mode needs more): three 512-thread blocks then fit a
// CU, so the 2M-agent build's ~740 buckets run in one round instead of ~1.4
// (bucket sort 42.8 -> 33.9 us on the sorted state).
// DEFER (large single builds): a bucket above the LDS stage does its counts,
// box starts and arrival slots here, then hands its chunks to k_sort_chunks
// (descriptors in `chunks`, capacity `cap`), so the chunks of the densest
// buckets are sorted by many blocks at once instead of one after another.
template <int M, bool GATHER, bool DEFER>
__global__ __launch_bounds__(kSortThreads)
__attribute__((amdgpu_waves_per_eu(6)))
void k_bucketsort(Header* __restrict__ hdr,
                                                             const int32_t* __restrict__ key2,
                                                             const int32_t* __restrict__ idx2,
                                                             const typename Mode<M>::Pay* __restrict__ pay2,
                                                             const typename Mode<M>::In* __restrict__ x,
                                                             const typename Mode<M>::In* __restrict__ y,
                                                             const typename Mode<M>::In* __restrict__ z,
                                                             const typename Mode<M>::In* __restrict__ d,
                                                             const int32_t* __restrict__ btot,
                                                             int32_t* __restrict__ start,
                                                             uint32_t* __restrict__ split,
                                                             int32_t* __restrict__ tmp,
                                                             int32_t* __restrict__ perm,
                                                             typename Mode<M>::Pay* __restrict__ pay,
                                                             uint2* __restrict__ payq,
                                                             const SimGeom* __restrict__ geom,
                                                             int32_t B, int4* __restrict__ chunks,
                                                             int32_t cap)
{
    __shared__ int32_t c[kSortBoxes];
    __shared__ int s_sims[2];
    __shared__ int32_t mem[kSortStage];      // input index of each box member, arrival order
    __shared__ uint8_t memq[kSortStage];     // its x-quarter
    __shared__ int32_t inv[kSortStage];      // final slot -> position in the bucket's input
    __shared__ int32_t s_wave[kSortThreads / kWave];
    if (hdr->error) return;
    const int b = blockIdx.x;
    if (b >= hdr->nb) return;
    const int sb = hdr->sb;
    const int64_t total = hdr->total_boxes;
    const int b0 = b << sb;
    const int nbox = (int)((total - b0) < (1ll << sb) ? (total - b0) : (1ll << sb));
    // bucket start: sum of the totals of the buckets before it
    int32_t part = 0;
    for (int k = threadIdx.x; k < b; k += kSortThreads) part += btot[k];
    part = wave_sum<int32_t>(part);
    if ((threadIdx.x & (kWave - 1)) == 0) s_wave[threadIdx.x / kWave] = part;
    __syncthreads();
    int32_t s0 = 0;
    for (int w = 0; w < kSortThreads / kWave; ++w) s0 += s_wave[w];
    __syncthreads();
    const int s1 = s0 + btot[b];
    const bool staged = (s1 - s0) <= kSortStage;   // block-uniform
    const PaySrc<M, GATHER> src{pay2, x, y, z, d};
    if (threadIdx.x == 0) {
        s_sims[0] = B > 1 ? sim_of_box(geom, B, b0) : 0;
        s_sims[1] = B > 1 ? sim_of_box(geom, B, b0 + (nbox > 0 ? nbox - 1 : 0)) : 0;
    }
    // 1. per-box counts
    for (int k = threadIdx.x; k < nbox; k += kSortThreads) c[k] = 0;
    __syncthreads();
    for (int e0 = s0 + threadIdx.x; e0 < s1; e0 += 4 * kSortThreads) {
        int kq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * kSortThreads;
            kq[u] = e < s1 ? key2[e] : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (kq[u] >= 0) atomicAdd(&c[kq[u] >> 2], 1);
    }
    __syncthreads();
    // 2. exclusive scan of the counts -> box starts (thread t owns a contiguous
    //    chunk); empty boxes get their (empty) split word here
    const int per = (nbox + kSortThreads - 1) / kSortThreads;
    const int k0 = threadIdx.x * per;
    int32_t sum = 0;
    for (int k = k0; k < k0 + per && k < nbox; ++k) sum += c[k];
    int32_t tot;
    int32_t run = block_excl_scan<kSortThreads, int32_t>(sum, s_wave, tot);
    for (int k = k0; k < k0 + per && k < nbox; ++k) {
        const int32_t v = c[k];
        c[k] = run;
        start[b0 + k] = s0 + run;
        if (v == 0) reinterpret_cast<uint2*>(split)[b0 + k] = make_uint2((uint32_t)(s0 + run), 0u);
        run += v;
    }
    __syncthreads();
    // 3. agents into their box range (arrival order)
    if (staged) {
        // at most U agents per thread: every load issued before the LDS work
        constexpr int U = kSortStage / kSortThreads;
        int kq[U], id[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = s0 + threadIdx.x + u * kSortThreads;
            kq[u] = e < s1 ? key2[e] : -1;
            id[u] = e < s1 ? idx2[e] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (kq[u] >= 0) {
                const int slot = atomicAdd(&c[kq[u] >> 2], 1);
                mem[slot] = id[u];
                memq[slot] = (uint8_t)(kq[u] & 3);
            }
        }
    } else {
        for (int e0 = s0 + threadIdx.x; e0 < s1; e0 += 4 * kSortThreads) {
            int kq[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * kSortThreads;
                kq[u] = e < s1 ? key2[e] : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (kq[u] >= 0) tmp[s0 + atomicAdd(&c[kq[u] >> 2], 1)] = e0 + u * kSortThreads - s0;
        }
    }
    __syncthreads();
    if (!staged) {   // block-uniform
        if constexpr (DEFER) {
            if (threadIdx.x == 0) {
                int cnt = 0;
                for (int kb = 0, cs = 0; kb < nbox; ++cnt) {
                    int ke, ce;
                    chunk_end(c, nbox, kb, cs, ke, ce);
                    kb = ke;
                    cs = ce;
                }
                const int base = (int)atomicAdd(&hdr->nchunk, (uint32_t)cnt);
                if (base + cnt > cap) {
                    atomicOr(&hdr->error, (uint32_t)ERR_CAPACITY);   // not reached: cap bounds it
                } else {
                    int i = base;
                    for (int kb = 0, cs = 0; kb < nbox; ++i) {
                        int ke, ce;
                        chunk_end(c, nbox, kb, cs, ke, ce);
                        chunks[2 * i] = make_int4(b, s0, kb, ke);
                        chunks[2 * i + 1] = make_int4(cs, ce, 0, 0);
                        kb = ke;
                        cs = ce;
                    }
                }
            }
        } else {
            sort_chunks<M, GATHER>(s0, nbox, b0, c, mem, memq, inv, key2, idx2, src, tmp, split,
                                   perm, pay, SlotQ(payq, geom, s_sims[0], s_sims[1]));
        }
        return;
    }
    // 4. c[k] now holds the end of box k.  Rank among box mates by (quarter,
    //    input index); the box's first agent in that order writes the split
    //    word (how many mates lie in quarters below 1, 2, 3).
    for (int e = s0 + threadIdx.x; e < s1; e += kSortThreads) {
        const int kq = key2[e];
        const int k = kq >> 2, q = kq & 3;
        const int32_t orig = idx2[e];
        const int bs = k > 0 ? c[k - 1] : 0;
        const int be = c[k];
        int r = 0;
        uint32_t w = 0;
        for (int m = bs; m < be; ++m) {
            const int qm = memq[m];
            r += (qm < q || (qm == q && mem[m] < orig)) ? 1 : 0;
            w += split_inc(qm);
        }
        if (r == 0)
            reinterpret_cast<uint2*>(split)[b0 + k] = make_uint2((uint32_t)(s0 + bs), split_word(w, be - bs));
        inv[bs + r] = e - s0;
    }
    __syncthreads();
    // 5. write the sorted bucket in slot order (loads issued before the stores)
    if (s1 > s0) {   // block-uniform; padding lanes read slot s0
        const SlotQ s32(payq, geom, s_sims[0], s_sims[1]);
        constexpr int UA = kSortStage / kSortThreads;
        // FP64 inputs are written in two halves, so that half as many 8-byte
        // values are in flight (fewer VGPRs, more blocks per CU)
        constexpr int HALVES = 2;
        constexpr int U = UA / HALVES;
        const int cnt = s1 - s0;
#pragma unroll
        for (int hh = 0; hh < HALVES; ++hh) {
            int e[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = threadIdx.x + (hh * U + u) * kSortThreads;
                e[u] = s0 + (p < cnt ? inv[p] : 0);
            }
            int32_t id[U], bx[U];
            typename Mode<M>::Pay q[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                id[u] = idx2[e[u]];
                bx[u] = b0 + (key2[e[u]] >> 2);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) q[u] = src.get(e[u], id[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = threadIdx.x + (hh * U + u) * kSortThreads;
                if (p < cnt) {
                    perm[s0 + p] = id[u];
                    pay[s0 + p] = q[u];
                    s32.put(s0 + p, q[u], bx[u]);
                }
            }
        }
    }
}

// The chunks handed over by a DEFER bucket sort (single simulation): each
// block takes descriptors i = blockIdx.x, + gridDim.x, ..., loads the
// chunk's box ends from the box starts and sorts it as the bucket sort would.
template <int M, bool GATHER>
__global__ __launch_bounds__(kSortThreads)
__attribute__((amdgpu_waves_per_eu(6)))
void k_sort_chunks(const Header* __restrict__ hdr, const int4* __restrict__ chunks, int32_t cap,
                   const int32_t* __restrict__ key2, const int32_t* __restrict__ idx2,
                   const typename Mode<M>::Pay* __restrict__ pay2,
                   const typename Mode<M>::In* __restrict__ x,
                   const typename Mode<M>::In* __restrict__ y,
                   const typename Mode<M>::In* __restrict__ z,
                   const typename Mode<M>::In* __restrict__ d,
                   const int32_t* __restrict__ start, uint32_t* __restrict__ split,
                   const int32_t* __restrict__ tmp, int32_t* __restrict__ perm,
                   typename Mode<M>::Pay* __restrict__ pay, uint2* __restrict__ payq,
                   const SimGeom* __restrict__ geom)
{
    __shared__ int32_t c[kSortBoxes];
    __shared__ int32_t mem[kSortStage];
    __shared__ uint8_t memq[kSortStage];
    __shared__ int32_t inv[kSortStage];
    if (hdr->error) return;
    const int nc = (int)hdr->nchunk < cap ? (int)hdr->nchunk : cap;
    const int sb = hdr->sb;
    const PaySrc<M, GATHER> src{pay2, x, y, z, d};
    const SlotQ s32(payq, geom, 0, 0);
    for (int i = blockIdx.x; i < nc; i += gridDim.x) {   // block-uniform
        const int4 d0 = chunks[2 * i], d1 = chunks[2 * i + 1];
        const int s0 = d0.y, kb = d0.z, ke = d0.w, cs = d1.x, ce = d1.y;
        const int b0 = d0.x << sb;
        // box ends relative to the bucket start, boxes kb - 1 .. ke - 1
        for (int k = kb - 1 + (int)threadIdx.x; k < ke; k += kSortThreads)
            if (k >= 0) c[k] = start[b0 + k + 1] - s0;
        __syncthreads();
        sort_chunk<M, GATHER>(s0, b0, kb, ke, cs, ce, c, mem, memq, inv, key2, idx2, src, tmp,
                              split, perm, pay, s32);
        __syncthreads();
    }
}

// ---------------------------------------------------------- canonical order

// The canonical order of the exports (ascending box, then input index) from
// the payload order (box, quarter, input index): each payload slot ranks its
// agent among the box's agents by input index.
__global__ __launch_bounds__(kBlock) void k_canon(int64_t n, const Header* __restrict__ hdr,
                                                  const int32_t* __restrict__ box_id,
                                                  const int32_t* __restrict__ start,
                                                  const int32_t* __restrict__ perm,
                                                  int32_t* __restrict__ canon,
                                                  int32_t* __restrict__ cslot)
{
    if (hdr->error) return;
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int32_t me = perm[k];
    const int32_t b = box_id[me];
    const int bs = start[b], be = start[b + 1];
    int r = 0;
    for (int m = bs; m < be; ++m) r += perm[m] < me ? 1 : 0;
    canon[bs + r] = me;
    cslot[bs + r] = (int32_t)k;
}

// The partition and the per-bucket sort, payload carried (GATHER false) or
// read from the inputs by the sort (GATHER true).
template <int M, bool GATHER>
void sort_passes(const Layout& L, const Dev& D, const typename Mode<M>::In* x,
                 const typename Mode<M>::In* y, const typename Mode<M>::In* z,
                 const typename Mode<M>::In* d, int64_t n, int32_t B, unsigned nba,
                 const int32_t* btot, hipStream_t s)
{
    using Pay = typename Mode<M>::Pay;
    if constexpr (sizeof(Pay) == sizeof(F4))
        k_partition_lds<M, GATHER><<<nba, kTileThreads, 0, s>>>(x, y, z, d, n, D.hdr, D.box_id,
                                                                D.quarter, D.hist, btot, D.key2,
                                                                D.idx2, static_cast<F4*>(D.pay2));
    else
        k_partition<M, GATHER><<<nba, kTileThreads, 0, s>>>(x, y, z, d, n, D.hdr, D.box_id,
                                                            D.quarter, D.hist, btot, D.key2, D.idx2,
                                                            static_cast<Pay*>(D.pay2));
    const int32_t cap = (int32_t)(2 * (L.max_agents / kSortStage + 1) + L.nb_cap);
    if (B == 1 && n > (int64_t)kGeomSplit * kBoundsChunk) {
        k_bucketsort<M, GATHER, true><<<(unsigned)L.nb_cap, kSortThreads, 0, s>>>(
            D.hdr, D.key2, D.idx2, static_cast<const Pay*>(D.pay2), x, y, z, d, btot, D.start,
            D.split, D.tmp, D.perm, static_cast<Pay*>(D.payload), D.payq,
            static_cast<const SimGeom*>(D.geom), B, D.chunks, cap);
        k_sort_chunks<M, GATHER><<<kSortChunkBlocks, kSortThreads, 0, s>>>(
            D.hdr, D.chunks, cap, D.key2, D.idx2, static_cast<const Pay*>(D.pay2), x, y, z, d,
            D.start, D.split, D.tmp, D.perm, static_cast<Pay*>(D.payload), D.payq,
            static_cast<const SimGeom*>(D.geom));
    } else {
        k_bucketsort<M, GATHER, false><<<(unsigned)L.nb_cap, kSortThreads, 0, s>>>(
            D.hdr, D.key2, D.idx2, static_cast<const Pay*>(D.pay2), x, y, z, d, btot, D.start,
            D.split, D.tmp, D.perm, static_cast<Pay*>(D.payload), D.payq,
            static_cast<const SimGeom*>(D.geom), B, D.chunks, cap);
    }
}

template <int M>
hipError_t grid_build_mode(const Layout& L, const Dev& D, const void* xv, const void* yv,
                           const void* zv, const void* dv, int64_t n, const int64_t* off,
                           int32_t B, double edge, const double* edges, bool sorted_input,
                           int order, hipStream_t s)
{
    using In = typename Mode<M>::In;
    const In* x = static_cast<const In*>(xv);
    const In* y = static_cast<const In*>(yv);
    const In* z = static_cast<const In*>(zv);
    const In* d = static_cast<const In*>(dv);
    const bool batched = off != nullptr;
    const int64_t* woff = nullptr;
    if (batched) {
        k_copy_offsets<<<(B + 1 + kBlock - 1) / kBlock, kBlock, 0, s>>>(off, D.off, B, n, D.hdr);
        woff = D.off;
    }
    const unsigned nbb = (unsigned)((n + kBoundsChunk - 1) / kBoundsChunk);
    auto a16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    const bool vec = a16(x) && a16(y) && a16(z) && a16(d);
    if (batched)
        k_bounds<M, true><<<nbb, kBlock, 0, s>>>(x, y, z, d, n, woff, B, D.bpart, false);
    else
        k_bounds<M, false><<<nbb, kBlock, 0, s>>>(x, y, z, d, n, nullptr, 1, D.bpart, vec);
    if (batched) {
        k_geometry<<<(B + 15) / 16, 1024, 0, s>>>(D.bpart, D.geom, woff, n, B, edge, edges);
        k_boxbase<<<1, 1024, 0, s>>>(D.hdr, D.geom, B, n, L.max_boxes, L.nb_cap, D.start);
    }
    const unsigned nba = (unsigned)((n + kTileA - 1) / kTileA);
    if (batched)
        k_hist<M, true, false><<<nba, kTileThreads, 0, s>>>(x, y, z, n, woff, B, D.geom, D.hdr, D.box_id,
                                                     D.quarter, D.hist, D.bpart, edge, L.max_boxes,
                                                     L.nb_cap, MS_BOX_ORDER_ROWS, D.start);
    else if (nbb > (unsigned)kGeomSplit) {
        k_geometry1<<<1, 1024, 0, s>>>(D.bpart, n, edge, L.max_boxes, L.nb_cap, order, D.geom,
                                       D.hdr, D.start);
        k_clear_hist<<<1024, kBlock, 0, s>>>(D.hdr, D.hist, (int32_t)nba);
        k_hist<M, false, true><<<nba, kTileThreads, 0, s>>>(x, y, z, n, nullptr, 1, D.geom, D.hdr,
                                                            D.box_id, D.quarter, D.hist, D.bpart,
                                                            edge, L.max_boxes, L.nb_cap, order,
                                                            D.start);
    } else
        k_hist<M, false, false><<<nba, kTileThreads, 0, s>>>(x, y, z, n, nullptr, 1, D.geom, D.hdr,
                                                             D.box_id, D.quarter, D.hist, D.bpart,
                                                             edge, L.max_boxes, L.nb_cap, order,
                                                             D.start);
    int32_t* btot = D.bstart + L.nb_cap + 1;
    k_rowscan<<<(unsigned)L.nb_cap, kBlock, 0, s>>>(D.hdr, D.hist, (int32_t)nba, btot);
    if (sorted_input)
        sort_passes<M, true>(L, D, x, y, z, d, n, B, nba, btot, s);
    else
        sort_passes<M, false>(L, D, x, y, z, d, n, B, nba, btot, s);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_init(const Layout& L, const Dev& D, hipStream_t s)
{
    (void)L;
    k_init<<<1, 64, 0, s>>>(D.hdr);
    return hipGetLastError();
}

hipError_t launch_error_copy(const Dev& D, int32_t* out, hipStream_t s)
{
    k_error_copy<<<1, 64, 0, s>>>(D.hdr, out);
    return hipGetLastError();
}

hipError_t launch_canon(const Layout& L, const Dev& D, int64_t n, hipStream_t s)
{
    (void)L;
    if (n <= 0) return hipSuccess;
    k_canon<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(n, D.hdr, D.box_id, D.start,
                                                                    D.perm, D.canon, D.cslot);
    return hipGetLastError();
}

hipError_t launch_grid_build(const Layout& L, const Dev& D, const void* x, const void* y,
                             const void* z, const void* d, int64_t n, const int64_t* off,
                             int32_t B, double edge, const double* edges, bool sorted_input,
                             int order, hipStream_t s)
{
    switch (L.dtype) {
    case MS_F32:
        return grid_build_mode<MS_F32>(L, D, x, y, z, d, n, off, B, edge, edges, sorted_input,
                                       order, s);
    case MS_F64:
        return grid_build_mode<MS_F64>(L, D, x, y, z, d, n, off, B, edge, edges, sorted_input,
                                       order, s);
    case MS_F32_POS64:
        return grid_build_mode<MS_F32_POS64>(L, D, x, y, z, d, n, off, B, edge, edges,
                                             sorted_input, order, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ms
