// Host side of the C ABI declared in include/mechstep.h: argument checks,
// workspace layout, kernel launches on the caller's stream.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <vector>

#include "launch.hpp"

namespace {

thread_local char g_err[512] = "";

ms_status fail(ms_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

ms_status ok()
{
    g_err[0] = '\0';
    return MS_OK;
}

ms_status check_hip(hipError_t e, const char* what)
{
    if (e != hipSuccess) return fail(MS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return ok();
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

size_t in_size(int dtype) { return dtype == MS_F32 ? 4 : 8; }     // positions, diameters
size_t out_size(int dtype) { return dtype == MS_F64 ? 8 : 4; }    // displacements, gradients

ms_status check_ws(const ms_workspace* ws, const char* who)
{
    if (!ws) return fail(MS_EINVAL, "%s: null workspace", who);
    if (!ws->base) return fail(MS_EINVAL, "%s: workspace has no device buffer", who);
    if (ws->dtype < MS_F32 || ws->dtype > MS_F32_POS64)
        return fail(MS_EINVAL, "%s: workspace dtype %d unknown", who, ws->dtype);
    const ms::Layout L = ms::make_layout(ws->max_agents, ws->max_boxes, ws->max_sims, ws->dtype);
    if (ws->bytes < L.total)
        return fail(MS_EINVAL, "%s: workspace holds %zu bytes, needs %zu", who, ws->bytes, L.total);
    return MS_OK;
}

ms_status check_params(const ms_params* p, const char* who)
{
    if (!p) return fail(MS_EINVAL, "%s: null params", who);
    const double v[5] = {p->kappa, p->gamma, p->dt, p->max_disp, p->adherence};
    for (double x : v)
        if (!std::isfinite(x)) return fail(MS_EINVAL, "%s: non-finite parameter", who);
    if (p->dt < 0 || p->max_disp < 0 || p->adherence < 0)
        return fail(MS_EINVAL, "%s: dt, max_disp and adherence must be >= 0", who);
    return MS_OK;
}

ms_status check_arrays(const char* who, size_t elem, std::initializer_list<const void*> ptrs)
{
    for (const void* p : ptrs) {
        if (!p) return fail(MS_EINVAL, "%s: null array", who);
        if (!aligned(p, elem)) return fail(MS_EINVAL, "%s: array not %zu-byte aligned", who, elem);
    }
    return MS_OK;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

size_t ms_workspace_bytes(int64_t max_agents, int64_t max_boxes, int32_t max_sims, ms_dtype dtype)
{
    if (max_agents < 0 || max_boxes < 0 || max_boxes > ms::kMaxBoxes || max_sims < 1) return 0;
    return ms::make_layout(max_agents, max_boxes, max_sims, dtype).total;
}

ms_status ms_workspace_init(ms_workspace* ws, void* base, size_t bytes, int64_t max_agents,
                            int64_t max_boxes, int32_t max_sims, ms_dtype dtype, void* stream)
{
    if (!ws) return fail(MS_EINVAL, "ms_workspace_init: null workspace");
    if (!base) return fail(MS_EINVAL, "ms_workspace_init: null buffer");
    if (!aligned(base, 256)) return fail(MS_EINVAL, "ms_workspace_init: buffer not 256-byte aligned");
    if (dtype < MS_F32 || dtype > MS_F32_POS64)
        return fail(MS_EINVAL, "ms_workspace_init: unknown dtype %d", (int)dtype);
    if (max_agents < 0 || max_agents >= 2147483647LL)
        return fail(MS_ECAPACITY, "ms_workspace_init: max_agents must be in [0, 2^31-1)");
    if (max_boxes < 1 || max_boxes > ms::kMaxBoxes)
        return fail(MS_ECAPACITY, "ms_workspace_init: max_boxes must be in [1, 2^25] (a build sorts "
                                  "at most 8192 buckets of 4096 boxes)");
    if (max_sims < 1 || max_sims > (1 << 24))
        return fail(MS_ECAPACITY, "ms_workspace_init: max_sims must be in [1, 2^24]");
    const uint64_t pay_bytes = (uint64_t)max_agents * (dtype == MS_F64 ? 32u : 16u);
    if (pay_bytes >= (1ull << 32))
        return fail(MS_ECAPACITY, "ms_workspace_init: max_agents too large for this dtype "
                                  "(sorted payload must stay below 4 GiB)");
    const ms::Layout L = ms::make_layout(max_agents, max_boxes, max_sims, dtype);
    if (bytes < L.total)
        return fail(MS_EINVAL, "ms_workspace_init: %zu bytes given, %zu needed", bytes, L.total);
    ws->base = base;
    ws->bytes = bytes;
    ws->max_agents = max_agents;
    ws->max_boxes = max_boxes;
    ws->max_sims = max_sims;
    ws->dtype = dtype;
    ws->n_agents = 0;
    ws->n_sims = 0;
    ws->built = 0;
    ws->keep_forces = 0;
    ws->gather_list = 0;
    ws->sorted_input = 0;
    ws->gather_block = 0;
    ws->box_order = MS_BOX_ORDER_AUTO;
    ws->gather_walk = MS_WALK_LANES;
    return check_hip(ms::launch_init(L, ms::resolve(L, base), as_stream(stream)), "ms_workspace_init");
}

static ms_status build_common(ms_workspace* ws, const void* x, const void* y, const void* z,
                              const void* d, int64_t n, const int64_t* off, int32_t B, double edge,
                              const double* edges, void* stream, const char* who)
{
    ms_status st = check_ws(ws, who);
    if (st) return st;
    if (n < 0) return fail(MS_EINVAL, "%s: n < 0", who);
    if (n > ws->max_agents) return fail(MS_ECAPACITY, "%s: n = %lld exceeds max_agents = %lld", who,
                                        (long long)n, (long long)ws->max_agents);
    if (B > ws->max_sims) return fail(MS_ECAPACITY, "%s: %d simulations exceed max_sims = %d", who, B,
                                      ws->max_sims);
    if (!std::isfinite(edge)) return fail(MS_EINVAL, "%s: non-finite edge", who);
    if (ws->box_order < MS_BOX_ORDER_AUTO || ws->box_order > MS_BOX_ORDER_TILES)
        return fail(MS_EINVAL, "%s: box_order = %d is not an ms_box_order", who, ws->box_order);
    if (n > 0) {
        st = check_arrays(who, in_size(ws->dtype), {x, y, z, d});
        if (st) return st;
    }
    if (off && !aligned(off, 8)) return fail(MS_EINVAL, "%s: sim_offsets not 8-byte aligned", who);
    if (edges && !aligned(edges, 8)) return fail(MS_EINVAL, "%s: edges not 8-byte aligned", who);
    ws->n_agents = n;
    ws->n_sims = B;
    ws->built = off ? 2 : 1;
    const bool sorted_input = ws->sorted_input != 0;
    ws->sorted_input = 0;
    if (n == 0) return ok();
    const ms::Layout L = ms::make_layout(ws->max_agents, ws->max_boxes, ws->max_sims, ws->dtype);
    return check_hip(ms::launch_grid_build(L, ms::resolve(L, ws->base), x, y, z, d, n, off, B, edge,
                                           edges, sorted_input, ws->box_order, as_stream(stream)),
                     who);
}

ms_status ms_grid_build(ms_workspace* ws, const void* x, const void* y, const void* z,
                        const void* d, int64_t n, double edge, void* stream)
{
    return build_common(ws, x, y, z, d, n, nullptr, 1, edge, nullptr, stream, "ms_grid_build");
}

ms_status ms_grid_build_batched(ms_workspace* ws, const void* x, const void* y, const void* z,
                                const void* d, const int64_t* sim_offsets, int32_t n_sims,
                                int64_t n_total, const double* edges, void* stream)
{
    if (!sim_offsets) return fail(MS_EINVAL, "ms_grid_build_batched: null sim_offsets");
    if (n_sims < 1) return fail(MS_EINVAL, "ms_grid_build_batched: n_sims < 1");
    return build_common(ws, x, y, z, d, n_total, sim_offsets, n_sims, 0.0, edges, stream,
                        "ms_grid_build_batched");
}

// Contact-list length and block size of the forward gather chosen by the
// workspace.
static int gather_list(const ms_workspace* ws)
{
    return ws->gather_list == ms::kLongList ? ms::kLongList : ms::kMaxContacts;
}

static int gather_block(const ms_workspace* ws)
{
    return ws->gather_block == ms::kBlock ? ms::kBlock : ms::kForceBlockSmall;
}

static bool gather_flat(const ms_workspace* ws) { return ws->gather_walk != MS_WALK_PLANES; }

static ms_status step_common(const ms_workspace* ws, int want_built, const char* who)
{
    ms_status st = check_ws(ws, who);
    if (st) return st;
    if (ws->gather_list != 0 && ws->gather_list != ms::kMaxContacts &&
        ws->gather_list != ms::kLongList)
        return fail(MS_EINVAL, "%s: gather_list must be 0, %d or %d", who, ms::kMaxContacts,
                    ms::kLongList);
    if (ws->gather_block != 0 && ws->gather_block != ms::kForceBlockSmall &&
        ws->gather_block != ms::kBlock)
        return fail(MS_EINVAL, "%s: gather_block must be 0, %d or %d", who, ms::kForceBlockSmall,
                    ms::kBlock);
    if (ws->gather_walk != MS_WALK_LANES && ws->gather_walk != MS_WALK_PLANES)
        return fail(MS_EINVAL, "%s: gather_walk must be %d or %d", who, MS_WALK_LANES,
                    MS_WALK_PLANES);
    if (ws->built != want_built)
        return fail(MS_EINVAL, "%s: workspace holds no %s grid build", who,
                    want_built == 1 ? "plain" : "batched");
    return MS_OK;
}

ms_status ms_mech_step(const ms_workspace* ws, const ms_params* p, void* dx, void* dy, void* dz,
                       void* stream)
{
    const char* who = "ms_mech_step";
    ms_status st = step_common(ws, 1, who);
    if (st) return st;
    if ((st = check_params(p, who))) return st;
    const int64_t n = ws->n_agents;
    if (n == 0) return ok();
    if ((st = check_arrays(who, out_size(ws->dtype), {dx, dy, dz}))) return st;
    const ms::Layout L = ms::make_layout(ws->max_agents, ws->max_boxes, ws->max_sims, ws->dtype);
    return check_hip(ms::launch_force(L, ms::resolve(L, ws->base), n, 1, false, p, nullptr, dx, dy,
                                      dz, nullptr, nullptr, nullptr, ws->keep_forces != 0,
                                      gather_list(ws), gather_block(ws), gather_flat(ws),
                                      as_stream(stream)),
                     who);
}

// Arguments of the fused step + position update: positions required, the
// displacement arrays all present or all null.
static ms_status check_step_integrate(const ms_workspace* ws, void* x, void* y, void* z, void* dx,
                                      void* dy, void* dz, const char* who)
{
    ms_status st = check_arrays(who, in_size(ws->dtype), {x, y, z});
    if (st) return st;
    const int nd = (dx != nullptr) + (dy != nullptr) + (dz != nullptr);
    if (nd != 0 && nd != 3) return fail(MS_EINVAL, "%s: dx, dy, dz must all be given or all NULL", who);
    if (nd == 3) return check_arrays(who, out_size(ws->dtype), {dx, dy, dz});
    return MS_OK;
}

ms_status ms_mech_step_integrate(const ms_workspace* ws, const ms_params* p, void* x, void* y,
                                 void* z, void* dx, void* dy, void* dz, void* stream)
{
    const char* who = "ms_mech_step_integrate";
    ms_status st = step_common(ws, 1, who);
    if (st) return st;
    if ((st = check_params(p, who))) return st;
    const int64_t n = ws->n_agents;
    if (n == 0) return ok();
    if ((st = check_step_integrate(ws, x, y, z, dx, dy, dz, who))) return st;
    const ms::Layout L = ms::make_layout(ws->max_agents, ws->max_boxes, ws->max_sims, ws->dtype);
    return check_hip(ms::launch_force(L, ms::resolve(L, ws->base), n, 1, false, p, nullptr, dx, dy,
                                      dz, x, y, z, ws->keep_forces != 0, gather_list(ws),
                                      gather_block(ws), gather_flat(ws),
                                      as_stream(stream)),
                     who);
}

// The sorted-state step: arguments checked, then the force kernel writes the
// state after the step in slot order.
static ms_status step_sorted_common(ms_workspace* ws, bool batched, const ms_params* p,
                                    const void* x, const void* y, const void* z, const void* d,
                                    void* xo, void* yo, void* zo, void* dout, void* dx, void* dy,
                                    void* dz, void* stream, const char* who)
{
    ms_status st = step_common(ws, batched ? 2 : 1, who);
    if (st) return st;
    if (batched) {
        if (!p || !aligned(p, 8)) return fail(MS_EINVAL, "%s: null or misaligned params", who);
    } else if ((st = check_params(p, who))) {
        return st;
    }
    const int64_t n = ws->n_agents;
    if (n == 0) return ok();
    const size_t ib = in_size(ws->dtype);
    if ((st = check_arrays(who, ib, {xo, yo, zo, dout}))) return st;
    const bool mixed = ws->dtype == MS_F32_POS64;
    if (mixed && (st = check_arrays(who, ib, {x, y, z, d}))) return st;
    const int nd = (dx != nullptr) + (dy != nullptr) + (dz != nullptr);
    if (nd != 0 && nd != 3) return fail(MS_EINVAL, "%s: dx, dy, dz must all be given or all NULL", who);
    if (nd == 3 && (st = check_arrays(who, out_size(ws->dtype), {dx, dy, dz}))) return st;
    // outputs must not overlap each other or the inputs
    const uintptr_t len = (uintptr_t)n * ib;
    const void* outs[4] = {xo, yo, zo, dout};
    const void* all[8] = {xo, yo, zo, dout, x, y, z, d};
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 8; ++b) {
            if (a == b || !all[b]) continue;
            const uintptr_t u = reinterpret_cast<uintptr_t>(outs[a]), v = reinterpret_cast<uintptr_t>(all[b]);
            if (u < v + len && v < u + len) return fail(MS_EINVAL, "%s: output arrays overlap", who);
        }
    ms::SortedState so{xo, yo, zo, dout, x, y, z, d};
    ws->sorted_input = 1;   // the state written in slot order feeds the next build
    const ms::Layout L = ms::make_layout(ws->max_agents, ws->max_boxes, ws->max_sims, ws->dtype);
    return check_hip(ms::launch_force(L, ms::resolve(L, ws->base), n, batched ? ws->n_sims : 1,
                                      batched, batched ? nullptr : p, batched ? p : nullptr, dx, dy,
                                      dz, nullptr, nullptr, nullptr,
                                      !batched && ws->keep_forces != 0, gather_list(ws),
                                      gather_block(ws), gather_flat(ws),
                                      as_stream(stream), &so),
                     who);
}

ms_status ms_mech_step_integrate_sorted(ms_workspace* ws, const ms_params* params,
                                        const void* x, const void* y, const void* z, const void* d,
                                        void* x_out, void* y_out, void* z_out, void* d_out,
                                        void* dx, void* dy, void* dz, void* stream)
{
    return step_sorted_common(ws, false, params, x, y, z, d, x_out, y_out, z_out, d_out, dx, dy, dz,
                              stream, "ms_mech_step_integrate_sorted");
}

ms_status ms_mech_step_batched_integrate_sorted(ms_workspace* ws, const ms_params* params,
                                                const void* x, const void* y, const void* z,
                                                const void* d, void* x_out, void* y_out,
                                                void* z_out, void* d_out, void* dx, void* dy,
                                                void* dz, void* stream)
{
    return step_sorted_common(ws, true, params, x, y, z, d, x_out, y_out, z_out, d_out, dx, dy, dz,
                              stream, "ms_mech_step_batched_integrate_sorted");
}

ms_status ms_mech_step_batched(const ms_workspace* ws, const ms_params* params, void* dx, void* dy,
                               void* dz, void* stream)
{
    const char* who = "ms_mech_step_batched";
    ms_status st = step_common(ws, 2, who);
    if (st) return st;
    if (!params || !aligned(params, 8)) return fail(MS_EINVAL, "%s: null or misaligned params", who);
    const int64_t n = ws->n_agents;
    if (n == 0) return ok();
    if ((st = check_arrays(who, out_size(ws->dtype), {dx, dy, dz}))) return st;
    const ms::Layout L = ms::make_layout(ws->max_agents, ws->max_boxes, ws->max_sims, ws->dtype);
    return check_hip(ms::launch_force(L, ms::resolve(L, ws->base), n, ws->n_sims, true, nullptr,
                                      params, dx, dy, dz, nullptr, nullptr, nullptr, false,
                                      gather_list(ws), gather_block(ws), gather_flat(ws),
                                      as_stream(stream)),
                     who);
}

ms_status ms_mech_step_batched_integrate(const ms_workspace* ws, const ms_params* params, void* x,
                                         void* y, void* z, void* dx, void* dy, void* dz,
                                         void* stream)
{
    const char* who = "ms_mech_step_batched_integrate";
    ms_status st = step_common(ws, 2, who);
    if (st) return st;
    if (!params || !aligned(params, 8)) return fail(MS_EINVAL, "%s: null or misaligned params", who);
    const int64_t n = ws->n_agents;
    if (n == 0) return ok();
    if ((st = check_step_integrate(ws, x, y, z, dx, dy, dz, who))) return st;
    const ms::Layout L = ms::make_layout(ws->max_agents, ws->max_boxes, ws->max_sims, ws->dtype);
    return check_hip(ms::launch_force(L, ms::resolve(L, ws->base), n, ws->n_sims, true, nullptr,
                                      params, dx, dy, dz, x, y, z, false, gather_list(ws),
                                      gather_block(ws), gather_flat(ws),
                                      as_stream(stream)),
                     who);
}

// acc: rollout mode (gdx..gdz are gx..gz, the position gradients in the
// positions' type, updated in place; gd and g_params are added to).
static ms_status backward_common(const ms_workspace* ws, bool batched, const ms_params* p,
                                 const void* gdx, const void* gdy, const void* gdz, void* gx,
                                 void* gy, void* gz, void* gd, double* g_params, bool acc,
                                 void* stream, const char* who)
{
    ms_status st = step_common(ws, batched ? 2 : 1, who);
    if (st) return st;
    if (batched) {
        if (!p || !aligned(p, 8)) return fail(MS_EINVAL, "%s: null or misaligned params", who);
    } else if ((st = check_params(p, who))) {
        return st;
    }
    if (!g_params || !aligned(g_params, 8)) return fail(MS_EINVAL, "%s: null g_params", who);
    const int64_t n = ws->n_agents;
    const ms::Layout L = ms::make_layout(ws->max_agents, ws->max_boxes, ws->max_sims, ws->dtype);
    if (n == 0) return ok();
    if ((st = check_arrays(who, acc ? in_size(ws->dtype) : out_size(ws->dtype),
                           {gdx, gdy, gdz, gx, gy, gz, gd})))
        return st;
    return check_hip(ms::launch_backward(L, ms::resolve(L, ws->base), n, batched ? ws->n_sims : 1,
                                         batched, batched ? nullptr : p, batched ? p : nullptr, gdx,
                                         gdy, gdz, gx, gy, gz, gd, g_params, gather_list(ws),
                                         gather_flat(ws), acc, as_stream(stream)),
                     who);
}

ms_status ms_mech_step_backward(const ms_workspace* ws, const ms_params* p, const void* gdx,
                                const void* gdy, const void* gdz, void* gx, void* gy, void* gz,
                                void* gd, double* g_params, void* stream)
{
    return backward_common(ws, false, p, gdx, gdy, gdz, gx, gy, gz, gd, g_params, false, stream,
                           "ms_mech_step_backward");
}

ms_status ms_mech_step_backward_accumulate(const ms_workspace* ws, const ms_params* p,
                                           void* pbx, void* pby, void* pbz, void* dbar,
                                           double* g_params, void* stream)
{
    return backward_common(ws, false, p, pbx, pby, pbz, pbx, pby, pbz, dbar, g_params, true, stream,
                           "ms_mech_step_backward_accumulate");
}

ms_status ms_mech_step_backward_batched(const ms_workspace* ws, const ms_params* params,
                                        const void* gdx, const void* gdy, const void* gdz, void* gx,
                                        void* gy, void* gz, void* gd, double* g_params,
                                        void* stream)
{
    return backward_common(ws, true, params, gdx, gdy, gdz, gx, gy, gz, gd, g_params, false, stream,
                           "ms_mech_step_backward_batched");
}

ms_status ms_mech_step_backward_batched_accumulate(const ms_workspace* ws, const ms_params* params,
                                                   void* pbx, void* pby, void* pbz, void* dbar,
                                                   double* g_params, void* stream)
{
    return backward_common(ws, true, params, pbx, pby, pbz, pbx, pby, pbz, dbar, g_params, true,
                           stream, "ms_mech_step_backward_batched_accumulate");
}

ms_status ms_integrate(void* x, void* y, void* z, const void* dx, const void* dy, const void* dz,
                       int64_t n, ms_dtype dtype, void* stream)
{
    const char* who = "ms_integrate";
    if (n < 0) return fail(MS_EINVAL, "%s: n < 0", who);
    if (dtype < MS_F32 || dtype > MS_F32_POS64) return fail(MS_EINVAL, "%s: unknown dtype", who);
    if (n == 0) return ok();
    ms_status st = check_arrays(who, in_size(dtype), {x, y, z});
    if (st) return st;
    if ((st = check_arrays(who, out_size(dtype), {dx, dy, dz}))) return st;
    return check_hip(ms::launch_integrate(x, y, z, dx, dy, dz, n, dtype, as_stream(stream)), who);
}

ms_status ms_reorder(ms_workspace* ws, const void* src, void* dst, int32_t elem_bytes,
                     void* stream)
{
    const char* who = "ms_reorder";
    ms_status st = check_ws(ws, who);
    if (st) return st;
    if (!ws->built) return fail(MS_EINVAL, "%s: no grid build", who);
    if (elem_bytes != 1 && elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8 && elem_bytes != 16)
        return fail(MS_EINVAL, "%s: elem_bytes must be 1, 2, 4, 8 or 16", who);
    const int64_t n = ws->n_agents;
    if (n == 0) return ok();
    if ((st = check_arrays(who, (size_t)elem_bytes, {src, dst}))) return st;
    const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
    const uintptr_t len = (uintptr_t)n * (uintptr_t)elem_bytes;
    if (a < b + len && b < a + len) return fail(MS_EINVAL, "%s: src and dst overlap", who);
    ws->sorted_input = 1;   // arrays renumbered into slot order feed the next build
    const ms::Layout L = ms::make_layout(ws->max_agents, ws->max_boxes, ws->max_sims, ws->dtype);
    return check_hip(ms::launch_reorder(ms::resolve(L, ws->base), n, src, dst, elem_bytes,
                                        as_stream(stream)),
                     who);
}

ms_status ms_grid_get(const ms_workspace* ws, ms_grid_info* info, int32_t* box_id,
                      int32_t* box_start, int32_t* perm, void* stream)
{
    const char* who = "ms_grid_get";
    ms_status st = check_ws(ws, who);
    if (st) return st;
    if (!ws->built) return fail(MS_EINVAL, "%s: no grid build", who);
    const ms::Layout L = ms::make_layout(ws->max_agents, ws->max_boxes, ws->max_sims, ws->dtype);
    const ms::Dev D = ms::resolve(L, ws->base);
    hipStream_t s = as_stream(stream);
    const int64_t n = ws->n_agents;
    const int32_t B = ws->n_sims;
    if (n == 0) {
        if (info) {
            for (int b = 0; b < B; ++b) {
                std::memset(&info[b], 0, sizeof(ms_grid_info));
            }
        }
        return ok();
    }
    ms::Header h;
    hipError_t e = hipMemcpyAsync(&h, D.hdr, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if ((st = check_hip(e, who))) return st;
    if (info) {
        std::vector<ms::SimGeom> g(B);
        std::vector<int64_t> off(B + 1);
        e = hipMemcpyAsync(g.data(), D.geom, sizeof(ms::SimGeom) * B, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && ws->built == 2)
            e = hipMemcpyAsync(off.data(), D.off, 8 * (B + 1), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if ((st = check_hip(e, who))) return st;
        if (ws->built == 1) { off[0] = 0; off[1] = n; }
        for (int b = 0; b < B; ++b) {
            ms_grid_info& I = info[b];
            for (int k = 0; k < 3; ++k) { I.origin[k] = g[b].origin[k]; I.dims[k] = g[b].dims[k]; }
            I.edge = g[b].edge;
            I.error = g[b].error | (int32_t)h.error;
            I.n_boxes = g[b].n_boxes;
            I.box_base = g[b].box_base;
            I.n_agents = off[b + 1] - off[b];
            I.tile_shift = g[b].tile_shift;
            I.reserved = 0;
        }
    }
    if (h.error) return fail(MS_EINVAL, "%s: the last build failed on the device (error bits %u)", who,
                             h.error);
    if (box_id) e = hipMemcpyAsync(box_id, D.box_id, 4 * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && box_start)
        e = hipMemcpyAsync(box_start, D.start, 4 * (h.total_boxes + 1), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && perm) e = ms::launch_canon(L, D, n, s);
    if (e == hipSuccess && perm) e = hipMemcpyAsync(perm, D.canon, 4 * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return check_hip(e, who);
}

ms_status ms_neighbors(const ms_workspace* ws, int32_t* counts, int64_t* offsets, int32_t* list,
                       int64_t cap, int64_t* total, void* stream)
{
    const char* who = "ms_neighbors";
    ms_status st = check_ws(ws, who);
    if (st) return st;
    if (!ws->built) return fail(MS_EINVAL, "%s: no grid build", who);
    if (!offsets || !aligned(offsets, 8)) return fail(MS_EINVAL, "%s: null offsets", who);
    const int64_t n = ws->n_agents;
    if (n > 0 && (!counts || !aligned(counts, 4))) return fail(MS_EINVAL, "%s: null counts", who);
    st = ms_device_status(ws, stream);
    if (st) return st;
    const ms::Layout L = ms::make_layout(ws->max_agents, ws->max_boxes, ws->max_sims, ws->dtype);
    const ms::Dev D = ms::resolve(L, ws->base);
    hipStream_t s = as_stream(stream);
    const bool batched = ws->built == 2;
    int64_t tot = 0;
    hipError_t e = hipSuccess;
    if (n == 0) {
        e = hipMemcpyAsync(offsets, &tot, 8, hipMemcpyHostToDevice, s);
    } else {
        e = ms::launch_canon(L, D, n, s);
        if (e == hipSuccess)
            e = ms::launch_neighbors_count(L, D, n, ws->n_sims, batched, counts, offsets, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&tot, offsets + n, 8, hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if ((st = check_hip(e, who))) return st;
    if (total) *total = tot;
    if (!list) return ok();
    if (cap < tot) return fail(MS_ECAPACITY, "%s: list holds %lld, needs %lld", who, (long long)cap,
                               (long long)tot);
    if (n == 0) return ok();
    if (!aligned(list, 4)) return fail(MS_EINVAL, "%s: list not aligned", who);
    e = ms::launch_neighbors_fill(L, D, n, ws->n_sims, batched, offsets, list, s);
    return check_hip(e, who);
}

ms_status ms_device_status(const ms_workspace* ws, void* stream)
{
    const char* who = "ms_device_status";
    ms_status st = check_ws(ws, who);
    if (st) return st;
    const ms::Layout L = ms::make_layout(ws->max_agents, ws->max_boxes, ws->max_sims, ws->dtype);
    const ms::Dev D = ms::resolve(L, ws->base);
    hipStream_t s = as_stream(stream);
    uint32_t err = 0;
    hipError_t e = hipSuccess;
    if (ws->built && ws->n_agents > 0) e = hipMemcpyAsync(&err, &D.hdr->error, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if ((st = check_hip(e, who))) return st;
    if (err & (ms::ERR_NONFINITE | ms::ERR_NEGDIAM))
        return fail(MS_EINPUT, "non-finite position/diameter or negative diameter (bits %u)", err);
    if (err & ms::ERR_CAPACITY)
        return fail(MS_ECAPACITY, "the grid needs more boxes than the workspace holds (max_boxes, "
                                  "at most 2^25) (bits %u)", err);
    if (err) return fail(MS_EINVAL, "edge or simulation offsets invalid (bits %u)", err);
    return ok();
}

ms_status ms_copy_probe(void* dst, const void* src, size_t bytes, void* stream)
{
    const char* who = "ms_copy_probe";
    if (!dst || !src || !aligned(dst, 16) || !aligned(src, 16) || bytes % 16)
        return fail(MS_EINVAL, "%s: pointers must be 16-byte aligned and bytes a multiple of 16", who);
    if (bytes == 0) return ok();
    return check_hip(ms::launch_copy_probe(dst, src, bytes, as_stream(stream)), who);
}

// ------------------------------------------------- the step without allocation

}  // extern "C"

namespace {

constexpr int64_t kNoAllocAgents = MS_NOALLOC_MAX_AGENTS;
constexpr int64_t kNoAllocBoxes = MS_NOALLOC_MAX_BOXES;
// The largest layout of the three modes (MS_F64 has 32-byte payloads).
constexpr size_t kNoAllocBytes = ms::make_layout(kNoAllocAgents, kNoAllocBoxes, 1, MS_F64).total;
static_assert(ms::make_layout(kNoAllocAgents, kNoAllocBoxes, 1, MS_F32).total <= kNoAllocBytes &&
                  ms::make_layout(kNoAllocAgents, kNoAllocBoxes, 1, MS_F32_POS64).total <=
                      kNoAllocBytes,
              "the static workspace holds every mode");

// The workspace of ms_mech_step_noalloc, one copy per GPU for the life of the
// process.  Host code never uses this name as an address: each device's copy
// is reached through the pointer hipGetSymbolAddress returns for it.
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // per device ordinal; null until first used

// Device address of the current device's scratch (looked up once per device).
ms_status scratch_address(void** out, const char* who)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(MS_EDEVICE, "%s: hipGetDevice: %s", who, hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MS_EDEVICE, "%s: hipGetSymbolAddress(scratch) on device %d: %s", who, dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MS_OK;
}

}  // namespace

extern "C" {

ms_status ms_mech_step_noalloc(const void* x, const void* y, const void* z, const void* d, int64_t n,
                               ms_dtype dtype, double edge, const ms_params* p, void* dx, void* dy,
                               void* dz, int32_t* dev_error, void* stream)
{
    const char* who = "ms_mech_step_noalloc";
    if (dtype < MS_F32 || dtype > MS_F32_POS64) return fail(MS_EINVAL, "%s: unknown dtype %d", who, (int)dtype);
    if (n < 0) return fail(MS_EINVAL, "%s: n < 0", who);
    if (n > kNoAllocAgents)
        return fail(MS_ECAPACITY, "%s: n = %lld exceeds MS_NOALLOC_MAX_AGENTS = %lld", who,
                    (long long)n, (long long)kNoAllocAgents);
    ms_status st = check_params(p, who);
    if (st) return st;
    if (!std::isfinite(edge)) return fail(MS_EINVAL, "%s: non-finite edge", who);
    if (dev_error && !aligned(dev_error, 4)) return fail(MS_EINVAL, "%s: dev_error not aligned", who);
    if (n > 0) {
        if ((st = check_arrays(who, in_size(dtype), {x, y, z, d}))) return st;
        if ((st = check_arrays(who, out_size(dtype), {dx, dy, dz}))) return st;
    }
    void* base = nullptr;
    if ((st = scratch_address(&base, who))) return st;
    hipStream_t s = as_stream(stream);
    const ms::Layout L = ms::make_layout(kNoAllocAgents, kNoAllocBoxes, 1, dtype);
    const ms::Dev D = ms::resolve(L, base);
    // a fresh header for every call: the array keeps the previous call's state
    hipError_t e = ms::launch_init(L, D, s);
    if (e == hipSuccess && n > 0)
        e = ms::launch_grid_build(L, D, x, y, z, d, n, nullptr, 1, edge, nullptr, false,
                                  MS_BOX_ORDER_AUTO, s);
    if (e == hipSuccess && n > 0)
        e = ms::launch_force(L, D, n, 1, false, p, nullptr, dx, dy, dz, nullptr, nullptr, nullptr,
                             false, ms::kMaxContacts, ms::kForceBlockSmall, true, s);
    if (e == hipSuccess && dev_error) e = ms::launch_error_copy(D, dev_error, s);
    return check_hip(e, who);
}

const char* ms_last_error(void) { return g_err; }

}  // extern "C"
