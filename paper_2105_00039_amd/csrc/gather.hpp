// Device building blocks of the 27-box gather (Section IV-A) and of the Eq. 1
// force (Section III), shared by the forward, backward and export kernels.
//
// Agents are stored in box-sorted order, boxes are numbered row-major with x
// fastest, so the 27 boxes around box (ix, iy, iz) are 9 contiguous runs of
// sorted slots: for each (dz, dy) the boxes ix-1 .. ix+1 of one x-row,
// clipped to the grid.  A run is [start[first box], start[last box + 1]).
#pragma once

#include "common.hpp"

#include <type_traits>

namespace ms {

// Fast single-precision square root / reciprocal (about 1 ulp), used on the
// FP32 path whose tolerance is far above their error.
__device__ __forceinline__ float fsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ float frcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double fsqrt(double v) { return sqrt(v); }
__device__ __forceinline__ double frcp(double v) { return 1.0 / v; }
// a / b: through the fast reciprocal on the FP32 path, exact on the FP64 path.
__device__ __forceinline__ float rdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double rdiv(double a, double b) { return a / b; }

// Simulation of every thread of a block over a sorted or input range:
// thread 0 finds the simulations of the block's first and last index, then
// each thread searches only between them.  s_range: two ints of LDS, free
// again when this returns (the gather kernels lend the first entries of
// their contact lists, so no extra LDS limits how many blocks fit a CU).
template <int NT = kBlock>
__device__ __forceinline__ int block_sim(const int64_t* __restrict__ off, int32_t B, int64_t n,
                                         int64_t first, int64_t i, int* s_range)
{
    if (threadIdx.x == 0) {
        const int64_t last = (first + NT < n ? first + NT : n) - 1;
        s_range[0] = find_sim(off, 0, B, first);
        s_range[1] = find_sim(off, 0, B, last);
    }
    __syncthreads();
    const int s = i < n ? find_sim(off, s_range[0], s_range[1] + 1, i) : 0;
    __syncthreads();
    return s;
}

struct Cell { int ix, iy, iz; };

// Materialise a loaded value at this point of the program.  The compiler
// otherwise sinks a load into the only branch that consumes it, which
// serialises loads meant to be in flight together.
__device__ __forceinline__ void pin4(uint32_t (&v)[4])
{
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]));
}
template <typename Pay>
__device__ __forceinline__ void pin4(Pay (&q)[4])
{
    asm volatile("" : "+v"(q[0].x), "+v"(q[0].y), "+v"(q[0].z), "+v"(q[0].w),
                      "+v"(q[1].x), "+v"(q[1].y), "+v"(q[1].z), "+v"(q[1].w),
                      "+v"(q[2].x), "+v"(q[2].y), "+v"(q[2].z), "+v"(q[2].w),
                      "+v"(q[3].x), "+v"(q[3].y), "+v"(q[3].z), "+v"(q[3].w));
}
__device__ __forceinline__ void pin(F4& q) { asm volatile("" : "+v"(q.x), "+v"(q.y), "+v"(q.z), "+v"(q.w)); }
__device__ __forceinline__ void pin(D4& q) { asm volatile("" : "+v"(q.x), "+v"(q.y), "+v"(q.z), "+v"(q.w)); }
__device__ __forceinline__ void pin(uint2& q) { asm volatile("" : "+v"(q.x), "+v"(q.y)); }

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

// Calls fn(j0, j1) for the 9 runs of the 27-box stencil in (dz, dy)
// lexicographic order (ascending box order for row-major rows), each run
// ascending in x.
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
            const int row = g.box_base + box_row(cy, cz, ny, g.tile_shift) * nx;
            fn(start[row + x0], start[row + x1 + 1]);
        }
    }
}


// Explicit fused multiply-add (a*b + c, one rounding).  The library is built
// without implicit contraction, so every fusion in the force arithmetic is
// written here and the same expression rounds the same way in every kernel
// that inlines it.
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Squared length of (ux, uy, uz).
template <typename Real>
__device__ __forceinline__ Real len2(Real ux, Real uy, Real uz)
{
    return fmad(uz, uz, fmad(ux, ux, uy * uy));
}

// Force of one listed pair (Eq. 1) added to a; nothing unless the spheres
// overlap (delta > 0) and the centres differ.  FP32: 1/l from rsq, rho from
// a reciprocal; coincident centres give rsq(0) = inf and a NaN delta, which
// fails delta > 0.  Each pair's term is rounded before it is added (multiply,
// then add): two pairs that mirror each other then cancel exactly, as the
// oracle's do (a fused multiply-add would leave the rounding error of the
// first product behind).
__device__ __forceinline__ void contact_force(const F4& pi, const F4& q, float kap, float gam,
                                              float& ax, float& ay, float& az)
{
    const float ux = pi.x - q.x, uy = pi.y - q.y, uz = pi.z - q.z;
    const float l2 = len2(ux, uy, uz);
    const float rs = pi.w + q.w;
    const float il = __builtin_amdgcn_rsqf(l2);
    const float delta = fmad(-l2, il, rs);
    if (delta > 0.0f) {
        const float rho = pi.w * q.w * __builtin_amdgcn_rcpf(rs);
        const float sv = fmad(kap, delta, -gam * __builtin_amdgcn_sqrtf(rho * delta));
        const float sl = sv * il;
        ax += sl * ux;
        ay += sl * uy;
        az += sl * uz;
    }
}

// 1/x and 1/sqrt(x) for x > 0 from the hardware estimates, each refined by
// two Newton steps (the error squares at every step), to within about one
// unit in the last place: the FP64 pair term is held to 1e-12 of its scale,
// not to correct rounding.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return r;
}
__device__ __forceinline__ double rsq_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * __builtin_fma(-h * y, y, 1.5);
    y = y * __builtin_fma(-h * y, y, 1.5);
    return y;
}

// FP64: the contact decision and delta from the correctly rounded |u| (so
// a touching pair gets exactly nothing, as in the oracle), the rest of the
// term from refined reciprocals: 1/l, 1/(r_i + r_j) and sqrt(rho delta).
__device__ __forceinline__ void contact_force(const D4& pi, const D4& q, double kap, double gam,
                                              double& ax, double& ay, double& az)
{
    const double ux = pi.x - q.x, uy = pi.y - q.y, uz = pi.z - q.z;
    const double l2 = len2(ux, uy, uz);
    const double rs = pi.w + q.w;
    const double l = sqrt(l2);
    const double delta = rs - l;
    if (delta > 0.0 && l2 > 0.0) {
        const double rho = pi.w * q.w * rcp_nr(rs);
        const double rd = rho * delta;
        const double sv = fmad(kap, delta, -gam * (rd * rsq_nr(rd)));
        const double sl = sv * rcp_nr(l);
        ax += sl * ux;
        ay += sl * uy;
        az += sl * uz;
    }
}

// The 9 runs of the stencil for the force sums, all bounds loaded up front
// (one memory round trip), trimmed to the agents the sphere of reach
// r_i + e/2 around the agent can touch: a partner is at most e/2 in radius
// (the edge is at least the largest diameter), so every contact lies inside
// it.  A (dy, dz) row whose y-z distance from the agent is >= reach is
// skipped.  Otherwise the row can only hold contacts with |x_j - x_i| < w,
// w = sqrt(reach^2 - yz^2): the run starts in the box holding x_i - w and
// ends in the box holding x_i + w, and inside those two boxes the agents of
// the quarters wholly outside the interval are dropped (a box's agents are
// ordered by x-quarter; the split word gives where each quarter begins).
// The row and box decisions are FP64 (offsets of the agent from its own box
// faces; reach carries a relative margin of 1e-9).  The quarters of the
// interval ends are located in FP32 with w widened by 1e-5 e, far above the
// FP32 error of those positions (< 2e-7 e), so no quarter holding a contact
// is ever dropped.  Out-of-range rows give empty runs.
struct Runs { int b[9], e[9]; };

template <typename Real>
__device__ __forceinline__ Runs stencil_runs(const SimGeom& g, Cell c,
                                             const int32_t* __restrict__ start,
                                             const uint32_t* __restrict__ split, Real px, Real py,
                                             Real pz, Real ri)
{
    const int nx = g.dims[0], ny = g.dims[1], nz = g.dims[2];
    const double e = g.edge;
    const double reach = ((double)ri + 0.5 * e) * (1.0 + 1e-9);
    const double r2 = reach * reach;
    // offsets of the agent from the lower (lo) and upper (hi) faces of its box
    const double lx = ((double)px - g.origin[0]) - c.ix * e, hx = e - lx;
    const double ly = ((double)py - g.origin[1]) - c.iy * e, hy = e - ly;
    const double lz = ((double)pz - g.origin[2]) - c.iz * e, hz = e - lz;
    const double lx2 = lx * lx, hx2 = hx * hx;
    const double dy2[3] = {ly * ly, 0.0, hy * hy};
    const double dz2[3] = {lz * lz, 0.0, hz * hz};
    const float ef = (float)e, c4 = 4.0f / ef, lxf = (float)lx, pad = 1e-5f * ef;
    // box_row of the 9 rows as the sum of a y part and a z part (the same
    // terms box_row adds); tile shift 0 gives iz*ny + iy
    // (unsigned: the rows at -1 wrap and are never used)
    const uint32_t ts = (uint32_t)g.tile_shift, tm = (1u << ts) - 1u;
    const uint32_t nty = ((uint32_t)ny + tm) >> ts;
    uint32_t ry[3], rz[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint32_t cy = (uint32_t)(c.iy + k - 1), cz = (uint32_t)(c.iz + k - 1);
        ry[k] = ((cy >> ts) << (2u * ts)) + (cy & tm);
        rz[k] = (((cz >> ts) * nty) << (2u * ts)) + ((cz & tm) << ts);
    }
    uint32_t i0[9], i1[9];
    int qa[9], qb[9];
    bool okr[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        const int cz = c.iz + r / 3 - 1, cy = c.iy + r % 3 - 1;
        const double yz = dz2[r / 3] + dy2[r % 3];
        const bool ok = cz >= 0 && cz < nz && cy >= 0 && cy < ny && yz < r2;
        const bool lo_prev = c.ix > 0 && lx2 + yz < r2;        // interval reaches box ix-1
        const bool hi_next = c.ix + 1 < nx && hx2 + yz < r2;   // interval reaches box ix+1
        const float w = __builtin_amdgcn_sqrtf((float)(r2 - yz)) + pad;
        // interval ends relative to the lower face of the box they are looked up in
        const float rlo = lxf - w + (lo_prev ? ef : 0.0f);
        const float rhi = lxf + w - (hi_next ? ef : 0.0f);
        const int ta = (int)floorf(rlo * c4), tb = (int)floorf(rhi * c4);
        const int row = g.box_base + (int)(ry[r % 3] + rz[r / 3]) * nx;
        okr[r] = ok;
        // Byte offsets of the two end boxes (32-bit, from a scalar base).
        // Out-of-range rows read box 0 (an empty run), so all loads are
        // unconditional and issue back to back.
        i0[r] = ok ? 4u * (uint32_t)(row + (lo_prev ? c.ix - 1 : c.ix)) : 0u;
        i1[r] = ok ? 4u * (uint32_t)(row + (hi_next ? c.ix + 1 : c.ix)) : 0u;
        qa[r] = ta < 0 ? 0 : (ta > 3 ? 3 : ta);
        qb[r] = tb < 0 ? 0 : (tb > 3 ? 3 : tb);
    }
    // (start, split word) of the two end boxes: one 8-byte load each.  The
    // run ends at the end box's start plus its count (byte 3 of its split
    // word), or at the next box's start when the word holds no count.
    uint2 pa[9], pb[9];
    const char* wbase = reinterpret_cast<const char*>(split);
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        pa[r] = *reinterpret_cast<const uint2*>(wbase + 2u * i0[r]);
        pb[r] = *reinterpret_cast<const uint2*>(wbase + 2u * i1[r]);
    }
    Runs R;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        const uint32_t wb = pb[r].y;
        int sb = (int)pb[r].x + (int)(wb >> 24);
        if (wb == kSplitNone) sb = start[i1[r] / 4u + 1u];
        const int b = (int)pa[r].x + split_skip(pa[r].y, qa[r]);
        const int en = sb - split_cut(wb, qb[r]);
        R.b[r] = b;
        R.e[r] = (okr[r] && en > b) ? en : b;
    }
    return R;
}

// Candidate test on the quantised slot copy the build writes
// (one 8-byte word pair per slot): x, y, z relative to the grid origin in
// units of e / kQuantScale, rounded down, each kept modulo 2^16, and the
// radius in the same units rounded up, stored negated.  A stencil candidate
// lies within two box edges of the agent on every axis, i.e. within 2^14
// quanta, so the 16-bit wrapped differences are the exact differences of the
// quantised coordinates; the squares are summed exactly in 32-bit integers
// by the packed 16-bit dot product (at most 3 * 2^28).  Each difference is
// within one quantum of the true difference times the scale, so every pair
// with |u| < r_i + r_j satisfies |u_q| < rq_i + rq_j + kQuantMargin: no pair
// in contact is rejected, and the kernel's own precision decides every
// accepted pair (delta > 0 in contact_force), so the contacts and their
// order, hence the sums, are the same as with an exact test.  The scan then
// loads 8 bytes per candidate instead of 16 (FP32) or 32 (FP64), and tests it
// with five packed-integer operations.
typedef short short2v __attribute__((ext_vector_type(2)));
typedef unsigned short ushort2v __attribute__((ext_vector_type(2)));

struct PreQ {
    const uint2* payq;
    uint32_t axy;   // the agent's own (x, y) quanta
    uint32_t azr;   // its z quanta and rq + kQuantMargin
};

// The PreQ of slot k: the agent's own quantised words.
__device__ __forceinline__ PreQ preq_of(const uint2* __restrict__ payq, int64_t k)
{
    const uint2 v = payq[k];
    const int rq = -(int)(int16_t)(v.y >> 16);
    PreQ r;
    r.payq = payq;
    r.axy = v.x;
    r.azr = (v.y & 0xffffu) | ((uint32_t)(rq + kQuantMargin) << 16);
    return r;
}

// |u_q|^2 < (rq_i + rq_j + kQuantMargin)^2 on the quantised words of a candidate.
__device__ __forceinline__ bool quant_hit(const PreQ& p, uint2 q)
{
    const ushort2v dxy = __builtin_bit_cast(ushort2v, p.axy) - __builtin_bit_cast(ushort2v, q.x);
    const ushort2v dzr = __builtin_bit_cast(ushort2v, p.azr) - __builtin_bit_cast(ushort2v, q.y);
    const short2v sxy = __builtin_bit_cast(short2v, dxy);
    const short2v szr = __builtin_bit_cast(short2v, dzr);   // (dz, R)
    const short2v nzr = szr * (short2v){1, -1};              // (dz, -R)
    int t = __builtin_amdgcn_sdot2(sxy, sxy, 0, false);
    t = __builtin_amdgcn_sdot2(szr, nzr, t, false);
    return t < 0;
}

// Visit the candidates of agent `pi` that may touch it, in canonical order,
// calling on_pair(offset, payload) for each candidate that passes the
// quantised test, which keeps every pair in contact (offset = byte offset of
// its payload, self_off that of the agent itself).  The caller's on_pair must
// still check delta > 0 and |u| > 0: it sees the agent itself, and the list
// is handed over in groups of four padded with the agent's own entry.
//
// Two phases keep the wavefront busy.  The scan walks the 9 trimmed runs;
// four candidates are loaded before any is tested (offsets clamped into the
// run, surplus tests masked), and each passing candidate's offset is appended
// to this lane's list in LDS (`lst`, stride NT, the block size) without
// branching (the
// slot is always written, the cursor advances on a hit).  The pair work then
// runs over the list, four payload loads in flight at a time.  The list is
// drained (by the whole wavefront at once) before a group of four could
// overflow any lane's list, so pairs are handed over in candidate order.
// Offsets are 32-bit: a workspace holds fewer than 2^32 payload bytes.
// The scan reads the quantised slot copy `pre`; the list holds copy offsets,
// scaled to payload offsets when drained.  `flat` (uniform over the launch)
// picks how the lanes walk their 9 runs; each lane meets its candidates in
// the same order either way, so the results are the same bit for bit.
template <typename Real, typename Pay, int LIST = kMaxContacts, int NT = kBlock, typename OnPair>
__device__ __forceinline__ void scan_contacts(const SimGeom& g, Cell c, const Pay& pi,
                                              uint32_t self_off,
                                              const int32_t* __restrict__ start,
                                              const uint32_t* __restrict__ split,
                                              const Pay* __restrict__ pay, uint32_t* lst,
                                              const PreQ& pre, bool flat, OnPair&& on_pair)
{
    constexpr uint32_t P = (uint32_t)sizeof(Pay);
    constexpr uint32_t PS = (uint32_t)sizeof(uint2);   // bytes per scanned candidate
    constexpr uint32_t SH = P == 32 ? 2u : 1u;         // copy offset -> payload offset
    static_assert(LIST % 4 == 0, "the list drains in groups of four");
    const char* base = reinterpret_cast<const char*>(pay);
    const char* sbase = reinterpret_cast<const char*>(pre.payq);
    int cnt = 0;
    auto drain = [&]() {
        for (int t = 0; t < cnt; t += 4) {
            uint32_t o[4];
            Pay q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t v = lst[(t + u) * NT];
                o[u] = (t + u < cnt) ? (v << SH) : self_off;
            }
            pin4(o);
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = *reinterpret_cast<const Pay*>(base + o[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) on_pair(o[u], q[u]);
        }
        cnt = 0;
    };
    auto test = [&](uint2 q, uint32_t off, bool live) {
        pin(q);
        lst[cnt * NT] = off;
        cnt += (int)(live & quant_hit(pre, q));
    };
    using SPay = uint2;
    const Runs R = stencil_runs<Real>(g, c, start, split, pi.x, pi.y, pi.z, pi.w);
    // one group of four candidates from `off` of a run ending at `end`.  The
    // scanned region has three spare entries after the last agent, so the
    // loads past a run's end stay inside it; those slots are masked out of
    // the test.
    auto group = [&](uint32_t off, uint32_t end) {
        const SPay q0 = *reinterpret_cast<const SPay*>(sbase + off);
        const SPay q1 = *reinterpret_cast<const SPay*>(sbase + off + PS);
        const SPay q2 = *reinterpret_cast<const SPay*>(sbase + off + 2 * PS);
        const SPay q3 = *reinterpret_cast<const SPay*>(sbase + off + 3 * PS);
        test(q0, off, true);
        test(q1, off + PS, off + PS < end);
        test(q2, off + 2 * PS, off + 2 * PS < end);
        test(q3, off + 3 * PS, off + 3 * PS < end);
    };
    if (flat) {
        // Each lane walks its own runs one after another, so a wavefront
        // takes as many steps as its busiest lane has groups in all 9 runs
        // together, not the sum over the runs of the busiest lane's groups
        // in each.  The non-empty runs wait at the top of the lane's list
        // (begin and end, two entries each, in stencil order); the hits fill
        // the list from the bottom, below the runs not taken yet.
        static_assert(LIST >= 2 * 9 + 4, "room for the runs and a group of four");
        int nr = 0;
#pragma unroll
        for (int r = 0; r < 9; ++r) nr += R.e[r] > R.b[r] ? 1 : 0;
        {
            int p = LIST - 2 * nr;
#pragma unroll
            for (int r = 0; r < 9; ++r) {
                if (R.e[r] > R.b[r]) {
                    lst[p * NT] = (uint32_t)R.b[r] * PS;
                    lst[(p + 1) * NT] = (uint32_t)R.e[r] * PS;
                    p += 2;
                }
            }
        }
        int left = nr;   // runs still waiting in the list
        uint32_t off = 0, end = 0;
        auto next_run = [&]() {
            if (left > 0) {
                const int p = LIST - 2 * left;
                off = lst[p * NT];
                end = lst[(p + 1) * NT];
                --left;
            }
        };
        next_run();
        while (__any(off < end)) {
            // the whole wave drains when any lane's next group could reach
            // its waiting runs: the lanes' drains run side by side
            if (__any(cnt > LIST - 4 - 2 * left)) drain();
            if (off < end) {
                group(off, end);
                off += 4 * PS;
                if (off >= end) next_run();
            }
        }
    } else {
        // The lanes take the z-planes together and walk the three runs of
        // a plane one after another: fewer steps than run by run, while the
        // lanes' loads stay within one plane of slots (on dense populations
        // the flat walk spreads them over all three and loses more to the
        // memory path than it saves in steps).
#pragma unroll
        for (int pz = 0; pz < 3; ++pz) {
            const uint32_t b0 = (uint32_t)R.b[3 * pz] * PS, e0 = (uint32_t)R.e[3 * pz] * PS;
            const uint32_t b1 = (uint32_t)R.b[3 * pz + 1] * PS, e1 = (uint32_t)R.e[3 * pz + 1] * PS;
            const uint32_t b2 = (uint32_t)R.b[3 * pz + 2] * PS, e2 = (uint32_t)R.e[3 * pz + 2] * PS;
            uint32_t off = b0, end = e0;
            int k = 0;
            auto advance = [&]() {
                if (off >= end && k == 0) { k = 1; off = b1; end = e1; }
                if (off >= end && k == 1) { k = 2; off = b2; end = e2; }
            };
            advance();
            while (__any(off < end)) {
                if (__any(cnt > LIST - 4)) drain();
                if (off < end) {
                    group(off, end);
                    off += 4 * PS;
                    advance();
                }
            }
        }
    }
    drain();
}

// Eq. 1 summed over every candidate in contact with agent `pi`, in canonical
// order (contact_force drops non-overlapping pairs and the agent itself).
// LIST: length of the per-lane contact list `lst` (stride NT, the block size).
template <typename Real, typename Pay, int LIST = kMaxContacts, int NT = kBlock>
__device__ __forceinline__ void force_sum(const SimGeom& g, Cell c, const Pay& pi,
                                          uint32_t self_off, const int32_t* __restrict__ start,
                                          const uint32_t* __restrict__ split,
                                          const Pay* __restrict__ pay, Real kap, Real gam,
                                          uint32_t* lst, const PreQ& pre, bool flat, Real& fx,
                                          Real& fy, Real& fz)
{
    Real ax = 0, ay = 0, az = 0;
    scan_contacts<Real, Pay, LIST, NT>(g, c, pi, self_off, start, split, pay, lst, pre, flat,
                                        [&](uint32_t, const Pay& q) {
        contact_force(pi, q, kap, gam, ax, ay, az);
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
