// Host-side launchers of the mechstep kernels (one translation unit each).
#pragma once

#include "common.hpp"

namespace ms {

// Clear the device state of a fresh workspace.
hipError_t launch_init(const Layout& L, const Dev& D, hipStream_t s);

// out[0] = the workspace's device error word (a one-thread kernel).
hipError_t launch_error_copy(const Dev& D, int32_t* out, hipStream_t s);

// Uniform grid: bounds -> geometry -> count -> scan -> scatter -> rank.
// off == nullptr means one simulation of n agents (B must be 1).
// sorted_input: the inputs are nearly box-sorted, the sort reads the payload
// from them (same build, different speed).  order: an ms_box_order, the row
// order of a single simulation's boxes (batched builds number rows
// row-major).
hipError_t launch_grid_build(const Layout& L, const Dev& D, const void* x, const void* y,
                             const void* z, const void* d, int64_t n, const int64_t* off,
                             int32_t B, double edge, const double* edges, bool sorted_input,
                             int order, hipStream_t s);

// Canonical order of the last build (ascending box, then input index) into
// D.canon / D.cslot, for the exports.
hipError_t launch_canon(const Layout& L, const Dev& D, int64_t n, hipStream_t s);

// Sorted-state step: the state after the step (positions + Delta and the
// diameters) written in the build's slot order to *_out; *_in are the build's
// inputs (read only in MS_F32_POS64 mode).
struct SortedState {
    void *x_out, *y_out, *z_out, *d_out;
    const void *x_in, *y_in, *z_in, *d_in;
};

// Forward step.  Single: p_host valid, off == nullptr.  Batched: p_dev valid.
// px/py/pz non-null: positions updated in place (p += Delta); dx/dy/dz may
// then be null.  sorted non-null: the sorted-state step (dx/dy/dz, if given,
// in slot order; px/py/pz unused).  keep (single only): also store the
// forces for the backward step.  list: contact-list length of the gather
// (kMaxContacts or kLongList); nt: threads per block of the gather
// (kForceBlockSmall or kBlock); flat: how the gather's lanes walk their runs
// (each lane all of its runs in turn, or the z-planes together; same results).
hipError_t launch_force(const Layout& L, const Dev& D, int64_t n, int32_t B, bool batched,
                        const ms_params* p_host, const ms_params* p_dev, void* dx, void* dy,
                        void* dz, void* px, void* py, void* pz, bool keep, int list, int nt,
                        bool flat, hipStream_t s, const SortedState* sorted = nullptr);

// Backward step; list, flat: contact-list length and run walk of its gathers
// (as launch_force).
// acc: rollout mode, gdx..gdz == gx..gz are the position gradients of the
// state type, updated in place (pbar += J^T pbar); gd and g_params are added to.
hipError_t launch_backward(const Layout& L, const Dev& D, int64_t n, int32_t B, bool batched,
                           const ms_params* p_host, const ms_params* p_dev, const void* gdx,
                           const void* gdy, const void* gdz, void* gx, void* gy, void* gz,
                           void* gd, double* g_params, int list, bool flat, bool acc,
                           hipStream_t s);

hipError_t launch_integrate(void* x, void* y, void* z, const void* dx, const void* dy,
                            const void* dz, int64_t n, int dtype, hipStream_t s);

// dst[k] = src[perm[k]] for the n slots of the last build (elem_bytes 1, 2, 4,
// 8 or 16).
hipError_t launch_reorder(const Dev& D, int64_t n, const void* src, void* dst, int elem_bytes,
                          hipStream_t s);

// Neighbour export: counts + offsets (phase 1), list (phase 2).
hipError_t launch_neighbors_count(const Layout& L, const Dev& D, int64_t n, int32_t B,
                                  bool batched, int32_t* counts, int64_t* offsets, hipStream_t s);
hipError_t launch_neighbors_fill(const Layout& L, const Dev& D, int64_t n, int32_t B,
                                 bool batched, const int64_t* offsets, int32_t* list,
                                 hipStream_t s);

// Gather of per-agent box ids in caller order for export.
hipError_t launch_copy_probe(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace ms
