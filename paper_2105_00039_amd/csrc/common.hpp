// Shared device/host definitions of the mechstep library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "mechstep.h"

namespace ms {

constexpr int kBlock = 256;           // threads per block for every per-agent kernel
constexpr int kWave = 64;             // CDNA wavefront
constexpr int kScanItems = 8;         // items per thread in the neighbour-offset scan
constexpr int kScanTile = kBlock * kScanItems;
constexpr int kBoundsChunk = kBlock * 16;   // agents per block in the bounds pass
constexpr int kTileThreads = 1024;    // threads per block of the bucket histogram/partition
constexpr int kTileA = 4096;          // agents per block in the bucket histogram/partition
constexpr int kBucketsMax = 8192;     // bucket count limit of the two-level sort
constexpr int kSBMin = 6;             // bucket = 2^SB consecutive boxes, SB in [6, 12]
constexpr int kSBMax = 12;
constexpr int kBucketAgents = 3072;   // target mean agents per bucket
constexpr int kSortThreads = 512;     // threads per block of the per-bucket sort
constexpr int kSortStage = 4096;      // buckets up to this many agents are sorted in LDS
constexpr int kMaxContacts = 24;      // per-lane contact list length of the gathers (default)
constexpr int kLongList = 40;         // the longer list the forward gather may use
constexpr int kForceBlockSmall = 64;  // the smaller block the forward gather may use
constexpr int kBwdBlock = 64;         // threads per block of the backward gather
constexpr int kRowTileShift = 4;      // tiled x-rows: 16 x 16 tiles of (iy, iz)
constexpr int64_t kTilePlaneAgents = 49152;   // agents per z-plane from which a build tiles its rows
// Quantised slot copy of plain builds (the gather's candidate test): quanta
// per box edge, and the margin (in quanta) added to the summed radii.
constexpr int kQuantScale = 8192;
constexpr int kQuantMargin = 2;
// Boxes a build can hold over all its simulations: the two-level sort keeps at
// most kBucketsMax buckets of at most 2^kSBMax boxes.
constexpr int64_t kMaxBoxes = (int64_t)kBucketsMax << kSBMax;
// The gather addresses each box's (start, split word) pair with a 32-bit byte
// offset of 8 bytes per box (two extra boxes past the last one).
static_assert((kMaxBoxes + 2) * 8 < (int64_t(1) << 32), "32-bit box-word offsets of the gather");

// Device error bits (ms_grid_info.error and the workspace error word).
enum : uint32_t {
    ERR_NONFINITE = 1u,   // non-finite position or diameter
    ERR_NEGDIAM = 2u,     // negative diameter
    ERR_EDGE = 4u,        // edge <= 0, non-finite, or below the largest diameter
    ERR_CAPACITY = 8u,    // more boxes than the workspace holds (at most kMaxBoxes)
    ERR_OFFSETS = 16u,    // simulation offsets do not partition [0, n)
};

// Workspace header (first 256 bytes of the device buffer).
struct Header {
    uint32_t error;        // error bits of the last build, rewritten by every build
    uint32_t n_sims;
    int32_t sb;            // bucket shift of the last build
    int32_t nb;            // bucket count of the last build
    int64_t total_boxes;   // boxes over all simulations of the last build
    int64_t n_agents;
    int64_t need_boxes;    // boxes the last build asked for (even when over capacity)
    uint32_t off_err;      // simulation-offset check of the current build (cleared after use)
    int32_t pad0;
    uint32_t build_gen;    // incremented by every build
    uint32_t fwd_gen;      // build_gen of the forward step that kept its forces
    ms_params fwd_params;  // parameters of that forward step
    uint32_t nchunk;       // chunk descriptors of the current large build's oversized buckets
    uint8_t pad[256 - 100];
};
static_assert(sizeof(Header) == 256, "header size");

// Per-simulation grid geometry (64 bytes).
struct SimGeom {
    double origin[3];
    double edge;
    int32_t dims[3];
    int32_t error;
    int32_t box_base;
    int32_t tile_shift;   // x-row numbering: 0 row-major, kRowTileShift tiled (box_row)
    int64_t n_boxes;
};
static_assert(sizeof(SimGeom) == 64, "geom size");

// Per-(block, simulation) bounds partial: min x,y,z, max x,y,z, max d, flags.
struct BoundsPart {
    double lo[3];
    double hi[3];
    double dmax;
    uint32_t flags;
    uint32_t pad;
};
static_assert(sizeof(BoundsPart) == 64, "bounds partial size");

struct alignas(16) F4 { float x, y, z, w; };
struct alignas(32) D4 { double x, y, z, w; };

template <int M> struct Mode;
template <> struct Mode<MS_F32>       { using In = float;  using Real = float;  using Pay = F4; };
template <> struct Mode<MS_F64>       { using In = double; using Real = double; using Pay = D4; };
template <> struct Mode<MS_F32_POS64> { using In = double; using Real = float;  using Pay = F4; };

// Byte offsets of every region of the workspace buffer.
struct Layout {
    size_t hdr, geom, off, bpart, box_id, quarter, start, split, hist, bstart, key2, idx2, pay2,
        tmp, perm, payload, payq, fbar, fsave, partials, scratch64, chunks, total;
    int64_t max_agents, max_boxes, n_part, nblk_a_max, nb_cap, nblk_b_max;
    int32_t max_sims;
    int32_t dtype;
};

constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

constexpr Layout make_layout(int64_t max_agents, int64_t max_boxes, int32_t max_sims,
                             int32_t dtype)
{
    Layout L{};
    L.max_agents = max_agents;
    L.max_boxes = max_boxes;
    L.max_sims = max_sims;
    L.dtype = dtype;
    const size_t pay = (dtype == MS_F64) ? sizeof(D4) : sizeof(F4);
    const int64_t na = max_agents > 0 ? max_agents : 1;
    const int64_t nblk = (na + kBlock - 1) / kBlock;
    L.nblk_a_max = (na + kTileA - 1) / kTileA;
    L.nblk_b_max = (na + kBoundsChunk - 1) / kBoundsChunk;
    int64_t nbc = (max_boxes + (1 << kSBMin) - 1) >> kSBMin;
    L.nb_cap = nbc < kBucketsMax ? (nbc > 0 ? nbc : 1) : kBucketsMax;
    L.n_part = (na + kBwdBlock - 1) / kBwdBlock + max_sims + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
    L.hdr = take(sizeof(Header));
    L.geom = take(sizeof(SimGeom) * (size_t)max_sims);
    L.off = take(8 * (size_t)(max_sims + 1));
    L.bpart = take(sizeof(BoundsPart) * (size_t)(L.nblk_b_max + max_sims + 1));
    L.box_id = take(4 * (size_t)na);
    L.quarter = take((size_t)na);
    L.start = take(4 * (size_t)(max_boxes + 2));
    L.split = take(8 * (size_t)(max_boxes + 2));
    L.hist = take(4 * (size_t)(L.nb_cap * L.nblk_a_max));
    L.bstart = take(4 * (size_t)(2 * L.nb_cap + 2));
    L.key2 = take(4 * (size_t)na);
    L.idx2 = take(4 * (size_t)na);
    L.pay2 = take(pay * (size_t)na);
    L.tmp = take(4 * (size_t)na);
    L.perm = take(4 * (size_t)na);
    // three extra entries: the gather reads up to three slots past a run's end
    L.payload = take(pay * (size_t)(na + 3));
    // an 8-byte quantised copy of each slot for the gather's candidate test
    // (same three extra entries)
    L.payq = take(8 * (size_t)(na + 3));
    L.fbar = take(pay * (size_t)na);
    L.fsave = take(pay * (size_t)na);
    L.partials = take(16 * (size_t)L.n_part);
    // int64 scratch for the neighbour-offset scan: one entry per scan tile of n+1 items
    L.scratch64 = take(8 * (size_t)((na + 1 + kScanTile - 1) / kScanTile + 1));
    // chunk descriptors of oversized buckets (32 bytes each): two consecutive
    // chunks of a bucket hold more than kSortStage agents, so a bucket has at
    // most 2 * agents / kSortStage + 1 of them
    L.chunks = take(32 * (size_t)(2 * (na / kSortStage + 1) + L.nb_cap));
    L.total = o;
    return L;
}

// Device pointers of every region.
struct Dev {
    Header* hdr;
    SimGeom* geom;
    int64_t* off;
    BoundsPart* bpart;
    int32_t* box_id;    // box index per agent, caller order
    uint8_t* quarter;   // x-quarter of each agent inside its box, caller order
    int32_t* start;     // box start offsets [total boxes + 1]
    uint32_t* split;    // per box b: [2b] = start[b], [2b + 1] = quarter split word
    int32_t* hist;      // [bucket][block-A] histogram, scanned in place along each row
    int32_t* bstart;    // [nb_cap+1 ...]: bucket totals
    int32_t* key2;      // build: (box in bucket) << 2 | quarter, bucket order
    int32_t* idx2;      // build: input index, bucket order
    void* pay2;
    int32_t* tmp;
    int32_t* perm;      // input index of each slot; slots ordered by (box, quarter, input index)
    // After a build key2 / idx2 are free; the exports reuse them for the
    // canonical order (box, input index): canon[c] = input index of canonical
    // slot c, cslot[c] = the payload slot holding it.
    int32_t* canon;
    int32_t* cslot;
    void* payload;
    uint2* payq;        // quantised (x, y | z, -r) of each slot (gather.hpp)
    void* fbar;
    void* fsave;        // forces of the last forward step that kept them (slot order)
    double* partials;
    long long* scratch64;
    int4* chunks;       // 2 per descriptor: (bucket, s0, kb, ke), (cs, ce, 0, 0)
};

inline Dev resolve(const Layout& L, void* base)
{
    char* b = static_cast<char*>(base);
    Dev d;
    d.hdr = reinterpret_cast<Header*>(b + L.hdr);
    d.geom = reinterpret_cast<SimGeom*>(b + L.geom);
    d.off = reinterpret_cast<int64_t*>(b + L.off);
    d.bpart = reinterpret_cast<BoundsPart*>(b + L.bpart);
    d.box_id = reinterpret_cast<int32_t*>(b + L.box_id);
    d.quarter = reinterpret_cast<uint8_t*>(b + L.quarter);
    d.start = reinterpret_cast<int32_t*>(b + L.start);
    d.split = reinterpret_cast<uint32_t*>(b + L.split);
    d.hist = reinterpret_cast<int32_t*>(b + L.hist);
    d.bstart = reinterpret_cast<int32_t*>(b + L.bstart);
    d.key2 = reinterpret_cast<int32_t*>(b + L.key2);
    d.idx2 = reinterpret_cast<int32_t*>(b + L.idx2);
    d.pay2 = b + L.pay2;
    d.tmp = reinterpret_cast<int32_t*>(b + L.tmp);
    d.perm = reinterpret_cast<int32_t*>(b + L.perm);
    d.canon = d.idx2;
    d.cslot = d.key2;
    d.payload = b + L.payload;
    d.payq = reinterpret_cast<uint2*>(b + L.payq);
    d.fbar = b + L.fbar;
    d.fsave = b + L.fsave;
    d.partials = reinterpret_cast<double*>(b + L.partials);
    d.scratch64 = reinterpret_cast<long long*>(b + L.scratch64);
    d.chunks = reinterpret_cast<int4*>(b + L.chunks);
    return d;
}

// ------------------------------------------------------------ device helpers

__device__ __forceinline__ unsigned long long enc_f64(double v)
{
    unsigned long long u = __double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ __forceinline__ double dec_f64(unsigned long long k)
{
    unsigned long long u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double(u);
}

// Number of the x-row (iy, iz) of a grid with ny rows along y.  Boxes are
// numbered x fastest (box = ix + nx * row), so the boxes of a row are
// contiguous whatever the row order.  s = 0: row-major, row = iz*ny + iy.
// s > 0: the rows are grouped in 2^s x 2^s tiles of (iy, iz), the tiles in
// row-major order (ceil(ny / 2^s) along y), and the rows row-major inside a
// tile; the tiles of the last column along y may be partly empty.
__host__ __device__ __forceinline__ int box_row(int iy, int iz, int ny, int s)
{
    const int m = (1 << s) - 1, nty = (ny + m) >> s;
    return ((((iz >> s) * nty + (iy >> s)) << (2 * s)) + ((iz & m) << s) + (iy & m));
}

// Box index along one axis: floor((p - o)/e) in FP64, clamped to [0, dim-1].
__device__ __forceinline__ int axis_index(double p, double o, double e, int dim)
{
    double q = floor((p - o) / e);
    int i = (q > 0.0) ? (int)q : 0;
    return i < dim - 1 ? i : dim - 1;
}

// Quarter of the box ix (along one axis) that holds coordinate p:
// floor(((p - o) - ix e) * (4/e)), clamped to [0, 3]; c4 = 4/e.  The grid
// build files every agent by it; the gather only needs it to within a small
// error, because it widens the bounds it looks up (see stencil_runs).
__device__ __forceinline__ int box_quarter(double p, double o, double c4, double e, int ix)
{
    const double t = floor(((p - o) - (double)ix * e) * c4);
    const int q = (t > 0.0) ? (int)t : 0;
    return q < 3 ? q : 3;
}

// The forces kept by a forward step are those of the backward's build and
// parameters.
__device__ __forceinline__ bool kept_forces_match(const Header* hdr, const ms_params& p)
{
    const ms_params& q = hdr->fwd_params;
    return hdr->fwd_gen == hdr->build_gen && q.kappa == p.kappa && q.gamma == p.gamma &&
           q.dt == p.dt && q.max_disp == p.max_disp && q.adherence == p.adherence;
}

// Per-box split word: bytes 0..2 hold the number of the box's agents in
// quarters below 1, 2, 3 (the slot offsets where quarters 1, 2, 3 begin), byte 3
// the box's agent count.  Boxes with more than 255 agents store kSplitNone and
// are not trimmed inside.
constexpr uint32_t kSplitNone = 0xffffffffu;

// Slots of box (word w) to skip at its start when the row interval begins in
// quarter q, and to drop at its end when it ends in quarter q.
__device__ __forceinline__ int split_skip(uint32_t w, int q)
{
    return (q == 0 || w == kSplitNone) ? 0 : (int)((w >> (8 * (q - 1))) & 0xffu);
}
__device__ __forceinline__ int split_cut(uint32_t w, int q)
{
    return (q == 3 || w == kSplitNone) ? 0 : (int)((w >> 24) - ((w >> (8 * q)) & 0xffu));
}

// Simulation owning index k of a concatenation with offsets off[0..B]:
// the largest s < B with off[s] <= k, searched in [lo, hi).
__device__ __forceinline__ int find_sim(const int64_t* __restrict__ off, int lo, int hi, int64_t k)
{
    // invariant: off[lo] <= k, answer in [lo, hi)
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid;
    }
    return lo;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) { T w = __shfl_xor(v, o); v = w < v ? w : v; }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) { T w = __shfl_xor(v, o); v = w > v ? w : v; }
    return v;
}

// Virtual block index that gives each XCD a contiguous share of the blocks.
// Work-groups are dispatched round-robin over the 8 XCDs, so block b runs on
// XCD b % 8; mapping those blocks to one contiguous range keeps the data that
// neighbouring virtual blocks share (candidate rows of the force gather,
// partially written cache lines of the partition's bucket runs) in the L2 of
// one XCD.
__device__ __forceinline__ unsigned xcd_block()
{
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned q = nb >> 3, r = nb & 7u, x = b & 7u;
    return x * q + (x < r ? x : r) + (b >> 3);
}

}  // namespace ms
