/*
 * mech_oracle.c -- plain, slow, FP64 CPU oracle for the mechanical-interaction
 * step of "GPU Acceleration of 3D Agent-Based Biological Simulations"
 * (arXiv 2105.00039).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The GPU product path never
 * links, imports or calls it, and this file shares no code with that path.
 *
 * Everything is computed in FP64, compiled without FMA contraction
 * (-ffp-contract=off) and without fast-math, one agent at a time, with every
 * sum taken in one fixed (canonical) order.
 *
 * What it computes (paper Section III, Eq. 1; Section IV-A, the uniform grid):
 *   1. A regular grid of cubic boxes of edge e over the agents' bounding box
 *      (Section IV-A: the simulation space is divided into equal voxels and
 *      each voxel holds the agents inside it; rebuilt every step).
 *   2. The neighbourhood of an agent: the agents of the 27 boxes around its own
 *      box (Section IV-A and its 2D figure of the 9 surrounding voxels).
 *   3. For every pair in contact (overlap delta > 0, Section III), the Eq. 1
 *      force  F = (kappa*delta - gamma*sqrt(rho*delta)) * (p1-p2)/|p1-p2|,
 *      delta = r1 + r2 - |p1-p2|, rho = r1*r2/(r1+r2), summed per agent.
 *   4. The displacement (Section III, end of the problem definition): no
 *      motion unless the force breaks the adherence; otherwise the force is
 *      integrated over the timestep and the displacement length is bounded.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - edge e: the caller's value, or the largest diameter when e <= 0; an edge
 *     below the largest diameter is rejected, so no contact can fall outside
 *     the 27 boxes.
 *   - origin = per-axis minimum, dims_k = floor((max_k - min_k)/e) + 1,
 *     box index ix = min(floor((x - o_x)/e), nx - 1), b = ix + nx*(iy + ny*iz)
 *     (row-major, x fastest).
 *   - within a box, agents are ordered by ascending input index; boxes by
 *     ascending index; so the 27-box stencil is visited in (dz, dy, dx)
 *     lexicographic order = ascending box index.  This is the canonical order.
 *   - contact iff delta > 0 (strict) and the centres differ (l > 0).
 *   - adherence a: the agent moves iff |F| > a.
 *   - integration: overdamped, v = dt*F; displacement = v if |v| <= m,
 *     else v*(m/|v|).
 *   - the exported neighbour set uses the predicate |p_i - p_j|^2 < e^2 with
 *     |u|^2 = (ux*ux + uy*uy) + uz*uz in FP64.
 *
 * Threads: built with OpenMP, the per-agent loops are split over threads.
 * Every agent's own sums stay sequential in canonical order and the global
 * sums (dL/dkappa, dL/dgamma) add per-agent partials in agent order, so the
 * results are identical bit for bit for any thread count.
 *
 * Status codes (same numbering as the product boundary so tests can compare
 * error behaviour): 0 ok, 1 invalid argument, 2 capacity, 4 invalid input
 * values (non-finite position/diameter or negative diameter).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ECAPACITY 2
#define ORC_EINPUT 4

typedef struct {
    double origin[3];
    double edge;
    int64_t dims[3];
    int64_t n_boxes;
} orc_geom;

/* ---------------------------------------------------------------- grid --- */

/* Bounding box, edge and box counts (Section IV-A; rebuilt every step). */
int orc_geometry(int64_t n, const double *x, const double *y, const double *z,
                 const double *d, double edge_in, double *origin3, double *edge_out,
                 int64_t *dims3, int64_t *n_boxes)
{
    if (n < 0) return ORC_EINVAL;
    if (!(edge_in == edge_in) || isinf(edge_in)) return ORC_EINVAL;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, dmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double p[3] = {x[i], y[i], z[i]};
        for (int k = 0; k < 3; ++k) {
            if (!isfinite(p[k])) return ORC_EINPUT;
            if (i == 0 || p[k] < lo[k]) lo[k] = p[k];
            if (i == 0 || p[k] > hi[k]) hi[k] = p[k];
        }
        if (!isfinite(d[i]) || d[i] < 0.0) return ORC_EINPUT;
        if (d[i] > dmax) dmax = d[i];
    }
    double e = edge_in > 0.0 ? edge_in : dmax;
    if (n > 0) {
        if (!(e > 0.0)) return ORC_EINVAL;   /* all diameters zero and no edge */
        if (e < dmax) return ORC_EINVAL;     /* a contact could escape the stencil */
    }
    int64_t nb = 1;
    for (int k = 0; k < 3; ++k) {
        int64_t dk = 1;
        if (n > 0) {
            double q = floor((hi[k] - lo[k]) / e);
            if (q >= 2147483646.0) return ORC_ECAPACITY;
            dk = (int64_t)q + 1;
        }
        dims3[k] = dk;
        origin3[k] = lo[k];
        nb *= dk;
        if (nb >= 2147483647LL) return ORC_ECAPACITY;
    }
    *edge_out = e;
    *n_boxes = (n > 0) ? nb : 0;
    return ORC_OK;
}

static int geom_of(int64_t n, const double *x, const double *y, const double *z,
                   const double *d, double edge_in, orc_geom *g)
{
    return orc_geometry(n, x, y, z, d, edge_in, g->origin, &g->edge, g->dims, &g->n_boxes);
}

static int64_t axis_index(double p, double o, double e, int64_t dim)
{
    int64_t i = (int64_t)floor((p - o) / e);
    if (i > dim - 1) i = dim - 1;
    if (i < 0) i = 0;
    return i;
}

static int64_t box_of(const orc_geom *g, double px, double py, double pz,
                      int64_t *ix, int64_t *iy, int64_t *iz)
{
    *ix = axis_index(px, g->origin[0], g->edge, g->dims[0]);
    *iy = axis_index(py, g->origin[1], g->edge, g->dims[1]);
    *iz = axis_index(pz, g->origin[2], g->edge, g->dims[2]);
    return *ix + g->dims[0] * (*iy + g->dims[1] * *iz);
}

/* Box index per agent, per-box start (exclusive prefix sum of the counts,
 * n_boxes + 1 entries) and the stable box-sorted order perm[slot] = agent.
 * Counting sort written out: count, exclusive scan, placement in ascending
 * agent index.  (Box::count and the per-box successor list of Section IV-A,
 * stored as contiguous segments.) */
static int build_grid(int64_t n, const double *x, const double *y, const double *z,
                      const orc_geom *g, int32_t *box_id, int32_t *start, int32_t *perm)
{
    int64_t nb = g->n_boxes;
    int64_t *cursor = (int64_t *)calloc((size_t)(nb > 0 ? nb : 1), sizeof(int64_t));
    if (!cursor) return ORC_EINVAL;
    for (int64_t b = 0; b <= nb; ++b) start[b] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t ix, iy, iz;
        int64_t b = box_of(g, x[i], y[i], z[i], &ix, &iy, &iz);
        box_id[i] = (int32_t)b;
        start[b + 1] += 1;                       /* count */
    }
    for (int64_t b = 0; b < nb; ++b) start[b + 1] += start[b];   /* exclusive scan */
    for (int64_t b = 0; b < nb; ++b) cursor[b] = start[b];
    for (int64_t i = 0; i < n; ++i) {            /* stable placement */
        int64_t b = box_id[i];
        perm[cursor[b]++] = (int32_t)i;
    }
    free(cursor);
    return ORC_OK;
}

int orc_grid(int64_t n, const double *x, const double *y, const double *z, const double *d,
             double edge_in, int32_t *box_id, int32_t *start, int32_t *perm)
{
    orc_geom g;
    int st = geom_of(n, x, y, z, d, edge_in, &g);
    if (st) return st;
    if (n == 0) { start[0] = 0; return ORC_OK; }
    return build_grid(n, x, y, z, &g, box_id, start, perm);
}

/* Internal: full grid in freshly allocated arrays. */
typedef struct {
    orc_geom g;
    int32_t *box_id, *start, *perm;
} orc_grid_t;

static void grid_free(orc_grid_t *G)
{
    free(G->box_id); free(G->start); free(G->perm);
}

static int grid_alloc_build(int64_t n, const double *x, const double *y, const double *z,
                            const double *d, double edge_in, orc_grid_t *G)
{
    memset(G, 0, sizeof(*G));
    int st = geom_of(n, x, y, z, d, edge_in, &G->g);
    if (st) return st;
    G->box_id = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    G->start = (int32_t *)malloc((size_t)(G->g.n_boxes + 1) * sizeof(int32_t));
    G->perm = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!G->box_id || !G->start || !G->perm) { grid_free(G); return ORC_EINVAL; }
    if (n == 0) { G->start[0] = 0; return ORC_OK; }
    return build_grid(n, x, y, z, &G->g, G->box_id, G->start, G->perm);
}

/* Visit the candidates of agent i in canonical order: stencil offsets
 * (dz, dy, dx) in {-1,0,1}^3 lexicographically, out-of-range boxes skipped,
 * agents of each box in ascending index, i itself excluded.  The callback
 * gets j.  Returns nothing; used by every pass below. */
typedef void (*visit_fn)(void *ctx, int64_t i, int64_t j);

static void visit_candidates(const orc_grid_t *G, const double *x, const double *y,
                             const double *z, int64_t i, visit_fn fn, void *ctx)
{
    int64_t ix, iy, iz;
    box_of(&G->g, x[i], y[i], z[i], &ix, &iy, &iz);
    const int64_t nx = G->g.dims[0], ny = G->g.dims[1], nz = G->g.dims[2];
    for (int dz = -1; dz <= 1; ++dz) {
        int64_t cz = iz + dz;
        if (cz < 0 || cz >= nz) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            int64_t cy = iy + dy;
            if (cy < 0 || cy >= ny) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                int64_t cx = ix + dx;
                if (cx < 0 || cx >= nx) continue;
                int64_t b = cx + nx * (cy + ny * cz);
                for (int64_t s = G->start[b]; s < G->start[b + 1]; ++s) {
                    int64_t j = G->perm[s];
                    if (j != i) fn(ctx, i, j);
                }
            }
        }
    }
}

/* ----------------------------------------------------------- neighbours --- */

static double dist2(double ux, double uy, double uz)
{
    return (ux * ux + uy * uy) + uz * uz;
}

typedef struct {
    const double *x, *y, *z;
    double e2;
    int64_t count;
    int32_t *out;       /* may be NULL */
} nb_ctx;

static void nb_visit(void *c, int64_t i, int64_t j)
{
    nb_ctx *C = (nb_ctx *)c;
    double ux = C->x[j] - C->x[i], uy = C->y[j] - C->y[i], uz = C->z[j] - C->z[i];
    if (dist2(ux, uy, uz) < C->e2) {
        if (C->out) C->out[C->count] = (int32_t)j;
        C->count += 1;
    }
}

/* Neighbour sets within the interaction radius e (Section III: every cell
 * interacts with all cells within a radius; Section IV-A: found through the
 * 27 surrounding boxes).  counts[i], offsets[n+1] (exclusive prefix of the
 * counts) and, if list != NULL and cap >= offsets[n], the lists themselves in
 * canonical order.  Returns ORC_ECAPACITY if list is given and too small. */
int orc_neighbors(int64_t n, const double *x, const double *y, const double *z,
                  const double *d, double edge_in, int32_t *counts, int64_t *offsets,
                  int32_t *list, int64_t cap)
{
    orc_grid_t G;
    int st = grid_alloc_build(n, x, y, z, d, edge_in, &G);
    if (st) { grid_free(&G); return st; }
    const double e2 = G.g.edge * G.g.edge;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        nb_ctx C = {x, y, z, e2, 0, NULL};
        visit_candidates(&G, x, y, z, i, nb_visit, &C);
        counts[i] = (int32_t)C.count;
    }
    offsets[0] = 0;
    for (int64_t i = 0; i < n; ++i) offsets[i + 1] = offsets[i] + counts[i];
    if (list) {
        if (cap < offsets[n]) { grid_free(&G); return ORC_ECAPACITY; }
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            nb_ctx C = {x, y, z, e2, 0, list + offsets[i]};
            visit_candidates(&G, x, y, z, i, nb_visit, &C);
        }
    }
    grid_free(&G);
    return ORC_OK;
}

/* O(N^2) brute force: for each i, every j != i in ascending index with
 * |p_j - p_i|^2 < R^2 (same FP64 expression).  Grid-free check of the sets. */
int orc_brute_neighbors(int64_t n, const double *x, const double *y, const double *z,
                        double R, int32_t *counts, int64_t *offsets, int32_t *list, int64_t cap)
{
    double R2 = R * R;
    offsets[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double ux = x[j] - x[i], uy = y[j] - y[i], uz = z[j] - z[i];
            if (dist2(ux, uy, uz) < R2) {
                if (list) {
                    if (offsets[i] + c >= cap) return ORC_ECAPACITY;
                    list[offsets[i] + c] = (int32_t)j;
                }
                ++c;
            }
        }
        counts[i] = (int32_t)c;
        offsets[i + 1] = offsets[i] + c;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- force --- */

/* Eq. 1 for one ordered pair (i, j): the force on i.  Adds to f[3] and
 * returns 1 if the pair is in contact. */
static int pair_force(double kappa, double gamma,
                      double xi, double yi, double zi, double ri,
                      double xj, double yj, double zj, double rj, double f[3])
{
    double ux = xi - xj, uy = yi - yj, uz = zi - zj;     /* p1 - p2 */
    double l = sqrt(dist2(ux, uy, uz));                  /* |p1 - p2| */
    double delta = (ri + rj) - l;                        /* overlap */
    if (!(delta > 0.0) || !(l > 0.0)) return 0;          /* not in contact */
    double rho = (ri * rj) / (ri + rj);                  /* combined radius */
    double s = kappa * delta - gamma * sqrt(rho * delta);
    double ex = ux / l, ey = uy / l, ez = uz / l;        /* unit direction */
    f[0] += s * ex;
    f[1] += s * ey;
    f[2] += s * ez;
    return 1;
}

typedef struct {
    const double *x, *y, *z, *d;
    double kappa, gamma;
    double f[3];
} force_ctx;

static void force_visit(void *c, int64_t i, int64_t j)
{
    force_ctx *C = (force_ctx *)c;
    pair_force(C->kappa, C->gamma, C->x[i], C->y[i], C->z[i], 0.5 * C->d[i],
               C->x[j], C->y[j], C->z[j], 0.5 * C->d[j], C->f);
}

/* Displacement from the total force (Section III): no motion if the force does
 * not exceed the adherence a; otherwise v = dt*F, bounded in length by m. */
static void displacement(const double F[3], double dt, double m, double a, double D[3])
{
    double fn = sqrt(dist2(F[0], F[1], F[2]));
    if (!(fn > a)) { D[0] = D[1] = D[2] = 0.0; return; }
    double v[3] = {dt * F[0], dt * F[1], dt * F[2]};
    double vn = sqrt(dist2(v[0], v[1], v[2]));
    if (vn > m) {
        double sc = m / vn;
        D[0] = v[0] * sc; D[1] = v[1] * sc; D[2] = v[2] * sc;
    } else {
        D[0] = v[0]; D[1] = v[1]; D[2] = v[2];
    }
}

static int check_params(const double *p)
{
    /* p = {kappa, gamma, dt, max_disp, adherence} */
    for (int k = 0; k < 5; ++k)
        if (!isfinite(p[k])) return ORC_EINVAL;
    if (p[2] < 0.0 || p[3] < 0.0 || p[4] < 0.0) return ORC_EINVAL;
    return ORC_OK;
}

/* One mechanical step: total force per agent (canonical order) and its
 * displacement.  fx..fz and dx..dz are [n] (any may be NULL). */
int orc_step(int64_t n, const double *x, const double *y, const double *z, const double *d,
             double edge_in, const double *params, double *fx, double *fy, double *fz,
             double *dx, double *dy, double *dz)
{
    int st = check_params(params);
    if (st) return st;
    orc_grid_t G;
    st = grid_alloc_build(n, x, y, z, d, edge_in, &G);
    if (st) { grid_free(&G); return st; }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        force_ctx C = {x, y, z, d, params[0], params[1], {0, 0, 0}};
        visit_candidates(&G, x, y, z, i, force_visit, &C);
        double D[3];
        displacement(C.f, params[2], params[3], params[4], D);
        if (fx) { fx[i] = C.f[0]; fy[i] = C.f[1]; fz[i] = C.f[2]; }
        if (dx) { dx[i] = D[0]; dy[i] = D[1]; dz[i] = D[2]; }
    }
    grid_free(&G);
    return ORC_OK;
}

/* O(N^2) brute-force force: Eq. 1 summed over every j != i in ascending index
 * (no grid, no radius).  Only the summation order differs from orc_step. */
int orc_brute_forces(int64_t n, const double *x, const double *y, const double *z,
                     const double *d, double kappa, double gamma,
                     double *fx, double *fy, double *fz)
{
    for (int64_t i = 0; i < n; ++i) {
        double f[3] = {0, 0, 0};
        for (int64_t j = 0; j < n; ++j)
            if (j != i)
                pair_force(kappa, gamma, x[i], y[i], z[i], 0.5 * d[i], x[j], y[j], z[j], 0.5 * d[j], f);
        fx[i] = f[0]; fy[i] = f[1]; fz[i] = f[2];
    }
    return ORC_OK;
}

/* ----------------------------------------------------- tolerance scales --- */

typedef struct {
    const double *x, *y, *z, *d;
    double kappa, gamma, u;
    double S, A;
    int64_t contacts;
} tol_ctx;

static void tol_visit(void *c, int64_t i, int64_t j)
{
    tol_ctx *C = (tol_ctx *)c;
    double ri = 0.5 * C->d[i], rj = 0.5 * C->d[j];
    double ux = C->x[i] - C->x[j], uy = C->y[i] - C->y[j], uz = C->z[i] - C->z[j];
    double l = sqrt(dist2(ux, uy, uz));
    double delta = (ri + rj) - l;
    double rho = (ri + rj) > 0.0 ? (ri * rj) / (ri + rj) : 0.0;
    double eta = 4.0 * C->u * (ri + rj + l);
    if (delta > 0.0 && l > 0.0) {
        C->S += C->kappa * delta + C->gamma * sqrt(rho * delta);
        C->contacts += 1;
    }
    if (delta > -eta) {
        double dm = delta > eta ? delta : eta;
        C->A += (C->kappa + C->gamma * sqrt(rho) / (2.0 * sqrt(dm))) * eta;
    }
}

/* Per-agent scales of the acceptance test used when comparing a force computed
 * in another precision or summation order with this oracle:
 *   S[i] = sum over contacts of (kappa*delta + gamma*sqrt(rho*delta))  (the
 *          magnitudes of both Eq. 1 terms, so cancellation inside s and across
 *          pairs cannot shrink the scale),
 *   A[i] = sum over pairs with delta > -eta of
 *          (kappa + gamma*sqrt(rho)/(2*sqrt(max(delta, eta)))) * eta,
 *          eta = 4u(ri + rj + l): the force a pair can carry when rounding of
 *          the distance flips its contact test,
 *   C[i] = number of contacts.
 * u is the unit roundoff of the compared precision. */
int orc_tolerance_scales(int64_t n, const double *x, const double *y, const double *z,
                         const double *d, double edge_in, double kappa, double gamma,
                         double u, double *S, double *A, int32_t *C)
{
    orc_grid_t G;
    int st = grid_alloc_build(n, x, y, z, d, edge_in, &G);
    if (st) { grid_free(&G); return st; }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        tol_ctx T = {x, y, z, d, kappa, gamma, u, 0, 0, 0};
        visit_candidates(&G, x, y, z, i, tol_visit, &T);
        S[i] = T.S; A[i] = T.A;
        if (C) C[i] = (int32_t)T.contacts;
    }
    grid_free(&G);
    return ORC_OK;
}

/* ------------------------------------------------------- sampled agents --- */
/*
 * The same per-agent results for a sample of agents only, for checks on
 * populations too large to evaluate whole: the grid is built over all n
 * agents (it is cheap), then orc_step's force and displacement and
 * orc_tolerance_scales' S, A, C are evaluated for the m agents idx[0..m) with
 * the very same per-agent code, so row k equals row idx[k] of the full
 * functions bit for bit.  Outputs are [m]; any output pointer may be NULL.
 */
int orc_sample(int64_t n, const double *x, const double *y, const double *z, const double *d,
               double edge_in, const double *params, double u, int64_t m, const int64_t *idx,
               double *fx, double *fy, double *fz, double *dx, double *dy, double *dz,
               double *S, double *A, int32_t *C)
{
    int st = check_params(params);
    if (st) return st;
    for (int64_t k = 0; k < m; ++k)
        if (idx[k] < 0 || idx[k] >= n) return ORC_EINVAL;
    orc_grid_t G;
    st = grid_alloc_build(n, x, y, z, d, edge_in, &G);
    if (st) { grid_free(&G); return st; }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < m; ++k) {
        const int64_t i = idx[k];
        force_ctx F = {x, y, z, d, params[0], params[1], {0, 0, 0}};
        tol_ctx T = {x, y, z, d, params[0], params[1], u, 0, 0, 0};
        visit_candidates(&G, x, y, z, i, force_visit, &F);
        double D[3];
        displacement(F.f, params[2], params[3], params[4], D);
        if (fx) { fx[k] = F.f[0]; fy[k] = F.f[1]; fz[k] = F.f[2]; }
        if (dx) { dx[k] = D[0]; dy[k] = D[1]; dz[k] = D[2]; }
        if (S || A || C) {
            visit_candidates(&G, x, y, z, i, tol_visit, &T);
            if (S) S[k] = T.S;
            if (A) A[k] = T.A;
            if (C) C[k] = (int32_t)T.contacts;
        }
    }
    grid_free(&G);
    return ORC_OK;
}

/* -------------------------------------------------------------- adjoint --- */
/*
 * Reverse-mode derivative of one step, derived from Eq. 1 and the
 * displacement rule.  Given gbar_i = dL/dDelta_i it returns
 *   gx,gy,gz[i] = sum_k (dDelta_k/dp_i)^T gbar_k,
 *   gd[i]       = sum_k (dDelta_k/dd_i)^T gbar_k,
 *   gkg[0..1]   = dL/dkappa, dL/dgamma.
 * (The identity term of p' = p + Delta is not included.)
 *
 * Step 1, displacement rule, per agent (F total force, v = dt F):
 *   |F| <= a          : Fbar = 0
 *   |v| <= m          : Fbar = dt * gbar
 *   otherwise         : Fbar = dt * (m/|v|) * (gbar - vhat (vhat . gbar))
 * Step 2, per contact pair (i, j) with e = (p_i - p_j)/l, s = kappa delta -
 * gamma sqrt(rho delta):
 *   ds/ddelta = kappa - gamma rho / (2 sqrt(rho delta)),
 *   ds/drho   = -gamma delta / (2 sqrt(rho delta)),
 *   drho/dr_i = r_j^2/(r_i + r_j)^2, ddelta/dr_i = 1, ddelta/dl = -1,
 *   d f_ij / d u = (s/l)(I - e e^T) - ds/ddelta e e^T  (symmetric),
 *   f_ji = -f_ij, so with w = Fbar_i - Fbar_j and q = e . w:
 *   pbar_i += (s/l)(w - e q) - ds/ddelta q e
 *   rbar_i += q (ds/ddelta + ds/drho r_j^2/(r_i + r_j)^2),  dbar_i = rbar_i/2
 *   kbar   += delta (e . Fbar_i),   gbar_gamma += -sqrt(rho delta)(e . Fbar_i)
 *   (the last two summed over ordered pairs, which counts each unordered pair
 *   once per side and gives delta q per pair).
 * Ties take the inactive branch: delta <= 0 is no contact, |v| = m is
 * unclamped, |F| = a is held.
 */
typedef struct {
    const double *x, *y, *z, *d;
    double kappa, gamma;
    const double *Fb;    /* [3n] */
    double pb[3], rb, kb, gb;
    double f[3];
} adj_ctx;

static void adj_force_visit(void *c, int64_t i, int64_t j)
{
    adj_ctx *C = (adj_ctx *)c;
    pair_force(C->kappa, C->gamma, C->x[i], C->y[i], C->z[i], 0.5 * C->d[i],
               C->x[j], C->y[j], C->z[j], 0.5 * C->d[j], C->f);
}

static void adj_visit(void *c, int64_t i, int64_t j)
{
    adj_ctx *C = (adj_ctx *)c;
    double ri = 0.5 * C->d[i], rj = 0.5 * C->d[j];
    double ux = C->x[i] - C->x[j], uy = C->y[i] - C->y[j], uz = C->z[i] - C->z[j];
    double l = sqrt(dist2(ux, uy, uz));
    double delta = (ri + rj) - l;
    if (!(delta > 0.0) || !(l > 0.0)) return;
    double rho = (ri * rj) / (ri + rj);
    double sq = sqrt(rho * delta);
    double s = C->kappa * delta - C->gamma * sq;
    double s_delta = C->kappa - C->gamma * rho / (2.0 * sq);
    double s_rho = -C->gamma * delta / (2.0 * sq);
    double e[3] = {ux / l, uy / l, uz / l};
    const double *Fi = C->Fb + 3 * i, *Fj = C->Fb + 3 * j;
    double w[3] = {Fi[0] - Fj[0], Fi[1] - Fj[1], Fi[2] - Fj[2]};
    double q = (e[0] * w[0] + e[1] * w[1]) + e[2] * w[2];
    for (int k = 0; k < 3; ++k)
        C->pb[k] += (s / l) * (w[k] - e[k] * q) - s_delta * q * e[k];
    double rs = ri + rj;
    C->rb += q * (s_delta + s_rho * (rj * rj) / (rs * rs));
    double eF = (e[0] * Fi[0] + e[1] * Fi[1]) + e[2] * Fi[2];
    C->kb += delta * eF;
    C->gb += -sq * eF;
}

/* Step 1 of the adjoint for every agent: the total force (canonical order)
 * pulled back through the displacement rule into Fb [3n]. */
static void fbar_all(const orc_grid_t *G, int64_t n, const double *x, const double *y,
                     const double *z, const double *d, const double *params,
                     const double *gdx, const double *gdy, const double *gdz, double *Fb)
{
    double dt = params[2], m = params[3], a = params[4];
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        adj_ctx C;
        memset(&C, 0, sizeof(C));
        C.x = x; C.y = y; C.z = z; C.d = d; C.kappa = params[0]; C.gamma = params[1];
        visit_candidates(G, x, y, z, i, adj_force_visit, &C);
        double g[3] = {gdx[i], gdy[i], gdz[i]};
        double fn = sqrt(dist2(C.f[0], C.f[1], C.f[2]));
        double *o = Fb + 3 * i;
        if (!(fn > a)) { o[0] = o[1] = o[2] = 0.0; continue; }
        double v[3] = {dt * C.f[0], dt * C.f[1], dt * C.f[2]};
        double vn = sqrt(dist2(v[0], v[1], v[2]));
        if (vn > m) {
            double vh[3] = {v[0] / vn, v[1] / vn, v[2] / vn};
            double vg = (vh[0] * g[0] + vh[1] * g[1]) + vh[2] * g[2];
            double sc = dt * (m / vn);
            for (int k = 0; k < 3; ++k) o[k] = sc * (g[k] - vh[k] * vg);
        } else {
            for (int k = 0; k < 3; ++k) o[k] = dt * g[k];
        }
    }
}

int orc_step_adjoint(int64_t n, const double *x, const double *y, const double *z,
                     const double *d, double edge_in, const double *params,
                     const double *gdx, const double *gdy, const double *gdz,
                     double *gx, double *gy, double *gz, double *gd, double *gkg)
{
    int st = check_params(params);
    if (st) return st;
    orc_grid_t G;
    st = grid_alloc_build(n, x, y, z, d, edge_in, &G);
    if (st) { grid_free(&G); return st; }
    double *Fb = (double *)calloc((size_t)(n > 0 ? 3 * n : 1), sizeof(double));
    double *kg = (double *)calloc((size_t)(n > 0 ? 2 * n : 1), sizeof(double));
    if (!Fb || !kg) { free(Fb); free(kg); grid_free(&G); return ORC_EINVAL; }
    fbar_all(&G, n, x, y, z, d, params, gdx, gdy, gdz, Fb);      /* step 1 */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {                             /* step 2 */
        adj_ctx C;
        memset(&C, 0, sizeof(C));
        C.x = x; C.y = y; C.z = z; C.d = d; C.kappa = params[0]; C.gamma = params[1]; C.Fb = Fb;
        visit_candidates(&G, x, y, z, i, adj_visit, &C);
        gx[i] = C.pb[0]; gy[i] = C.pb[1]; gz[i] = C.pb[2];
        gd[i] = 0.5 * C.rb;
        kg[2 * i] = C.kb; kg[2 * i + 1] = C.gb;
    }
    double kb = 0.0, gb = 0.0;
    for (int64_t i = 0; i < n; ++i) { kb += kg[2 * i]; gb += kg[2 * i + 1]; }
    gkg[0] = kb; gkg[1] = gb;
    free(Fb);
    free(kg);
    grid_free(&G);
    return ORC_OK;
}

/* ------------------------------------------------ gradient tolerance scales --- */
/*
 * Per-agent scales of the acceptance test used when comparing a gradient
 * computed in another precision or summation order with orc_step_adjoint.
 * Every term of the adjoint gather is linear in w = Fbar_i - Fbar_j with
 * coefficients built from s, ds/ddelta and ds/drho, so, with
 * W = |Fbar_i| + |Fbar_j| (which bounds |w| and |q| = |e . w| and cannot
 * cancel), summed over the contacts of agent i:
 *   Sp[i] = sum W (2|s|/l + |s_delta|)
 *           bounds |pbar_i| term by term: |(s/l)(w - e q)| <= (|s|/l)(|w| + |q|)
 *           and |s_delta q e| <= |s_delta| W;
 *   Sd[i] = sum W (|s_delta| + |s_rho| r_j^2/(r_i + r_j)^2) / 2, the same for dbar_i;
 *   Ap[i], Ad[i]: what rounding the overlap by eta = 4u(r_i + r_j + l) can
 *           change in them, eta times the derivatives in delta of the
 *           coefficients:
 *           Ap: sum eta W (2|s_delta|/l + s_dd),
 *           Ad: sum eta W (s_dd + gamma/(4 sqrt(rho dm)) r_j^2/(r_i + r_j)^2) / 2,
 *           s_dd = gamma rho^2 / (4 (rho dm)^(3/2)) = d s_delta / d delta,
 *           dm = max(delta, eta);
 *   skg[0..3] = {sum |delta| |Fbar_i|, sum eta |Fbar_i|,
 *                sum sqrt(rho delta) |Fbar_i|, sum eta rho/(2 sqrt(rho dm)) |Fbar_i|}
 *           over all ordered contact pairs: the scale and allowance of
 *           dL/dkappa, then of dL/dgamma.
 * Fbar is step 1 of orc_step_adjoint for the same gbar.  u is the unit
 * roundoff of the compared precision.
 */
typedef struct {
    const double *x, *y, *z, *d, *Fb;
    double kappa, gamma, u;
    double Sp, Ap, Sd, Ad, sk[4];
} adjtol_ctx;

static double norm3(const double *v) { return sqrt(dist2(v[0], v[1], v[2])); }

static void adjtol_visit(void *c, int64_t i, int64_t j)
{
    adjtol_ctx *C = (adjtol_ctx *)c;
    double ri = 0.5 * C->d[i], rj = 0.5 * C->d[j];
    double ux = C->x[i] - C->x[j], uy = C->y[i] - C->y[j], uz = C->z[i] - C->z[j];
    double l = sqrt(dist2(ux, uy, uz));
    double delta = (ri + rj) - l;
    if (!(delta > 0.0) || !(l > 0.0)) return;
    double rs = ri + rj;
    double rho = (ri * rj) / rs;
    double sq = sqrt(rho * delta);
    const double s = C->kappa * delta - C->gamma * sq;
    const double s_delta = C->kappa - C->gamma * rho / (2.0 * sq);
    const double s_rho = -(C->gamma * delta) / (2.0 * sq);
    const double eta = 4.0 * C->u * (ri + rj + l);
    double dm = delta > eta ? delta : eta;
    double sqm = sqrt(rho * dm);
    double s_dd = C->gamma * rho * rho / (4.0 * sqm * sqm * sqm);
    double c2 = (rj * rj) / (rs * rs);
    double fi = norm3(C->Fb + 3 * i), fj = norm3(C->Fb + 3 * j);
    double W = fi + fj;
    C->Sp += W * (2.0 * fabs(s) / l + fabs(s_delta));
    C->Ap += eta * W * (2.0 * fabs(s_delta) / l + s_dd);
    C->Sd += 0.5 * W * (fabs(s_delta) + fabs(s_rho) * c2);
    C->Ad += 0.5 * eta * W * (s_dd + C->gamma / (4.0 * sqm) * c2);
    C->sk[0] += delta * fi;
    C->sk[1] += eta * fi;
    C->sk[2] += sq * fi;
    C->sk[3] += eta * rho / (2.0 * sqm) * fi;
}

int orc_adjoint_scales(int64_t n, const double *x, const double *y, const double *z,
                       const double *d, double edge_in, const double *params,
                       const double *gdx, const double *gdy, const double *gdz, double u,
                       double *Sp, double *Ap, double *Sd, double *Ad, double *skg)
{
    int st = check_params(params);
    if (st) return st;
    orc_grid_t G;
    st = grid_alloc_build(n, x, y, z, d, edge_in, &G);
    if (st) { grid_free(&G); return st; }
    double *Fb = (double *)calloc((size_t)(n > 0 ? 3 * n : 1), sizeof(double));
    double *sk = (double *)calloc((size_t)(n > 0 ? 4 * n : 1), sizeof(double));
    if (!Fb || !sk) { free(Fb); free(sk); grid_free(&G); return ORC_EINVAL; }
    fbar_all(&G, n, x, y, z, d, params, gdx, gdy, gdz, Fb);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        adjtol_ctx C;
        memset(&C, 0, sizeof(C));
        C.x = x; C.y = y; C.z = z; C.d = d; C.Fb = Fb;
        C.kappa = params[0]; C.gamma = params[1]; C.u = u;
        visit_candidates(&G, x, y, z, i, adjtol_visit, &C);
        Sp[i] = C.Sp; Ap[i] = C.Ap; Sd[i] = C.Sd; Ad[i] = C.Ad;
        for (int k = 0; k < 4; ++k) sk[4 * i + k] = C.sk[k];
    }
    for (int k = 0; k < 4; ++k) skg[k] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 4; ++k) skg[k] += sk[4 * i + k];
    free(Fb);
    free(sk);
    grid_free(&G);
    return ORC_OK;
}

/* Threads of the OpenMP build for the calls that follow (ignored without
 * OpenMP); returns the number in use. */
int orc_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
    return omp_get_max_threads();
#else
    (void)t;
    return 1;
#endif
}

/* p <- p + Delta for every agent at once (Jacobi update). */
int orc_integrate(int64_t n, double *x, double *y, double *z,
                  const double *dx, const double *dy, const double *dz)
{
    for (int64_t i = 0; i < n; ++i) { x[i] += dx[i]; y[i] += dy[i]; z[i] += dz[i]; }
    return ORC_OK;
}

int orc_abi_version(void) { return 1; }
