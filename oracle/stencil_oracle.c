/*
 * stencil_oracle.c -- plain, slow, obviously correct FP64 reference of the
 * time-stepped stencil sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or helper with the
 * GPU path.
 *
 * What it computes (paper: Sec. 2.1, Alg. 1 "Heat-2D Stencil", Eq. 3):
 * every cell of a d-dimensional grid is replaced, once per time step, by a
 * weighted sum of itself and a fixed set of neighbours taken from the
 * previous step; two buffers alternate between steps (the A[t%2] / A[(t+1)%2]
 * double buffer of Alg. 1).  Readings of points the paper leaves open:
 *   - "for t = 0 -> T" runs exactly T steps (t = 0 .. T-1), matching the
 *     factor T in the stencils-per-second metric (Eq. 5);
 *   - the grid's shape is the number of updated cells; a neighbour index
 *     outside the grid reads 0 (zero-Dirichlet ghost layer, BC_ZERO) or wraps
 *     modulo the extent (BC_PERIODIC);
 *   - IEEE double, round to nearest, no fused multiply-add (build with
 *     -ffp-contract=off), points summed in the order given.
 *
 * The outflow (oracle_sweep_flux) is not in the paper either: it is the
 * bookkeeping of the zero rule read as an absorbing boundary -- a step moves
 * w_p * u(c) from cell c to the cell that reads c through point p, and what
 * would land outside the grid is counted as having left (summed in FP64).
 *
 * The variable-coefficient heat step and its adjoint are not in the paper;
 * they follow the conservative face-averaged form stated at
 * oracle_varcoef_step below, and the adjoint is the plain reverse-mode
 * derivative of that same loop (a scatter, independent of the fact that the
 * operator happens to be symmetric).
 *
 * Layout: dense C order, shape (nz, ny, nx) (leading axes of extent 1 for
 * 1D/2D), x unit-stride.  Offsets are npoints x ndim, slowest axis first.
 * All functions return 0 on success and a negative value on bad arguments.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_BC_ZERO 0
#define OR_BC_PERIODIC 1

typedef struct {
    int64_t n[3];      /* nz, ny, nx */
    int64_t cells;
} or_grid;

static int or_setup(int32_t ndim, const int64_t* shape, or_grid* g)
{
    if (ndim < 1 || ndim > 3 || shape == NULL) return -1;
    g->n[0] = g->n[1] = g->n[2] = 1;
    for (int d = 0; d < ndim; ++d) {
        if (shape[d] < 1) return -1;
        g->n[3 - ndim + d] = shape[d];
    }
    g->cells = g->n[0] * g->n[1] * g->n[2];
    return 0;
}

/* Read cell (z, y, x) of `a` under the boundary rule: an out-of-range index
 * reads 0 (zero rule) or wraps modulo the extent (periodic rule). */
static double or_read(const double* a, const or_grid* g, int32_t bc,
                      int64_t z, int64_t y, int64_t x)
{
    int64_t c[3] = {z, y, x};
    for (int d = 0; d < 3; ++d) {
        if (c[d] < 0 || c[d] >= g->n[d]) {
            if (bc == OR_BC_ZERO) return 0.0;
            c[d] %= g->n[d];
            if (c[d] < 0) c[d] += g->n[d];
        }
    }
    return a[(c[0] * g->n[1] + c[1]) * g->n[2] + c[2]];
}

static int or_threads(int32_t nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

int oracle_max_threads(void)
{
    return or_threads(0);
}

/* Weighted-sum form of Alg. 1:
 *   u_new[c] = sum_p w[p] * u[c + off[p]]   (p in the order given)
 * `u` holds u_0 on entry and u_T on exit. */
int oracle_sweep(int32_t ndim, const int64_t* shape, int32_t npoints,
                 const int32_t* offsets, const double* weights, int32_t bc,
                 int64_t steps, double* u, int32_t nthreads)
{
    or_grid g;
    if (or_setup(ndim, shape, &g) || npoints < 1 || !offsets || !weights || !u ||
        steps < 0 || (bc != OR_BC_ZERO && bc != OR_BC_PERIODIC))
        return -1;
    int32_t* off = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)npoints);
    double* other = (double*)malloc(sizeof(double) * (size_t)g.cells);
    if (!off || !other) { free(off); free(other); return -2; }
    for (int32_t p = 0; p < npoints; ++p) {
        off[3 * p + 0] = off[3 * p + 1] = off[3 * p + 2] = 0;
        for (int d = 0; d < ndim; ++d) off[3 * p + 3 - ndim + d] = offsets[p * ndim + d];
    }
    double* src = u;
    double* dst = other;
    const int nt = or_threads(nthreads);
    for (int64_t t = 0; t < steps; ++t) {
#pragma omp parallel for num_threads(nt) schedule(static)
        for (int64_t z = 0; z < g.n[0]; ++z)
            for (int64_t y = 0; y < g.n[1]; ++y)
                for (int64_t x = 0; x < g.n[2]; ++x) {
                    double acc = 0.0;
                    for (int32_t p = 0; p < npoints; ++p)
                        acc += weights[p] * or_read(src, &g, bc, z + off[3 * p],
                                                    y + off[3 * p + 1], x + off[3 * p + 2]);
                    dst[(z * g.n[1] + y) * g.n[2] + x] = acc;
                }
        double* tmp = src; src = dst; dst = tmp;
    }
    if (src != u) memcpy(u, src, sizeof(double) * (size_t)g.cells);
    free(off);
    free(other);
    return 0;
}

/* Transposed operator of oracle_sweep, applied `steps` times: every cell
 * scatters w[p] * v[c] to the cell that read it, c + off[p] (wrapped; dropped
 * when it falls on the zero ghost layer).  This is the adjoint of the
 * weighted-sum step written as the literal transpose, not as a mirrored
 * stencil, so it pins the mirrored-offset implementation independently. */
int oracle_sweep_transpose(int32_t ndim, const int64_t* shape, int32_t npoints,
                           const int32_t* offsets, const double* weights, int32_t bc,
                           int64_t steps, double* v)
{
    or_grid g;
    if (or_setup(ndim, shape, &g) || npoints < 1 || !offsets || !weights || !v ||
        steps < 0 || (bc != OR_BC_ZERO && bc != OR_BC_PERIODIC))
        return -1;
    double* out = (double*)malloc(sizeof(double) * (size_t)g.cells);
    if (!out) return -2;
    for (int64_t t = 0; t < steps; ++t) {
        memset(out, 0, sizeof(double) * (size_t)g.cells);
        for (int64_t z = 0; z < g.n[0]; ++z)
            for (int64_t y = 0; y < g.n[1]; ++y)
                for (int64_t x = 0; x < g.n[2]; ++x) {
                    const double vc = v[(z * g.n[1] + y) * g.n[2] + x];
                    for (int32_t p = 0; p < npoints; ++p) {
                        int64_t c[3] = {z, y, x};
                        int ghost = 0;
                        for (int d = 0; d < ndim; ++d) c[3 - ndim + d] += offsets[p * ndim + d];
                        for (int d = 0; d < 3; ++d) {
                            if (c[d] < 0 || c[d] >= g.n[d]) {
                                if (bc == OR_BC_ZERO) { ghost = 1; break; }
                                c[d] %= g.n[d];
                                if (c[d] < 0) c[d] += g.n[d];
                            }
                        }
                        if (!ghost) out[(c[0] * g.n[1] + c[1]) * g.n[2] + c[2]] += weights[p] * vc;
                    }
                }
        memcpy(v, out, sizeof(double) * (size_t)g.cells);
    }
    free(out);
    return 0;
}

/* Explicit heat step in its increment form, as the workloads state it:
 *   u_new = u + alpha * (sum of the 2*ndim axis neighbours - 2*ndim*u)
 * (Eq. 3 with mu = alpha, rearranged).  Neighbours are summed axis by axis,
 * slowest axis first, the -1 neighbour before the +1 neighbour. */
int oracle_heat(int32_t ndim, const int64_t* shape, double alpha, int32_t bc,
                int64_t steps, double* u, int32_t nthreads)
{
    or_grid g;
    if (or_setup(ndim, shape, &g) || !u || steps < 0 ||
        (bc != OR_BC_ZERO && bc != OR_BC_PERIODIC))
        return -1;
    double* other = (double*)malloc(sizeof(double) * (size_t)g.cells);
    if (!other) return -2;
    double* src = u;
    double* dst = other;
    const int nt = or_threads(nthreads);
    const double twod = 2.0 * ndim;
    for (int64_t t = 0; t < steps; ++t) {
#pragma omp parallel for num_threads(nt) schedule(static)
        for (int64_t z = 0; z < g.n[0]; ++z)
            for (int64_t y = 0; y < g.n[1]; ++y)
                for (int64_t x = 0; x < g.n[2]; ++x) {
                    int64_t c[3] = {z, y, x};
                    double s = 0.0;
                    for (int d = 3 - ndim; d < 3; ++d) {
                        for (int sg = -1; sg <= 1; sg += 2) {
                            int64_t q[3] = {c[0], c[1], c[2]};
                            q[d] += sg;
                            s += or_read(src, &g, bc, q[0], q[1], q[2]);
                        }
                    }
                    const double uc = src[(z * g.n[1] + y) * g.n[2] + x];
                    dst[(z * g.n[1] + y) * g.n[2] + x] = uc + alpha * (s - twod * uc);
                }
        double* tmp = src; src = dst; dst = tmp;
    }
    if (src != u) memcpy(u, src, sizeof(double) * (size_t)g.cells);
    free(other);
    return 0;
}

/* Value of one cell after `steps` weighted-sum steps, computed on the cone
 * of cells it depends on: the region needed shrinks by the stencil radius
 * per step, so a sample of a large run costs O(steps^(d+1)) instead of a full
 * sweep.  Same rules and summation order as oracle_sweep; equal to it up to
 * nothing (each computed cell is the identical expression).  `u0` is the full
 * initial field. */
int oracle_sweep_point(int32_t ndim, const int64_t* shape, int32_t npoints,
                       const int32_t* offsets, const double* weights, int32_t bc,
                       int64_t steps, const double* u0, const int64_t* at, double* out)
{
    or_grid g;
    if (or_setup(ndim, shape, &g) || npoints < 1 || !offsets || !weights || !u0 || !at ||
        !out || steps < 0 || (bc != OR_BC_ZERO && bc != OR_BC_PERIODIC))
        return -1;
    int32_t off[125 * 3];
    if (npoints > 125) return -1;
    int32_t rad = 0;
    for (int32_t p = 0; p < npoints; ++p) {
        off[3 * p + 0] = off[3 * p + 1] = off[3 * p + 2] = 0;
        for (int d = 0; d < ndim; ++d) {
            int32_t o = offsets[p * ndim + d];
            off[3 * p + 3 - ndim + d] = o;
            if (o > rad) rad = o;
            if (-o > rad) rad = -o;
        }
    }
    int64_t c[3] = {0, 0, 0};
    for (int d = 0; d < ndim; ++d) {
        c[3 - ndim + d] = at[d];
        if (at[d] < 0 || at[d] >= shape[d]) return -1;
    }
    /* Local window: cells c + [-h, h] on each real axis (h = rad*steps), held
     * as unwrapped coordinates; reads resolve through the boundary rule. */
    const int64_t h = (int64_t)rad * steps;
    int64_t lo[3], ext[3];
    for (int d = 0; d < 3; ++d) {
        const int real = d >= 3 - ndim;
        lo[d] = real ? c[d] - h : c[d];
        ext[d] = real ? 2 * h + 1 : 1;
    }
    const int64_t wcells = ext[0] * ext[1] * ext[2];
    double* a = (double*)malloc(sizeof(double) * (size_t)wcells);
    double* b = (double*)malloc(sizeof(double) * (size_t)wcells);
    if (!a || !b) { free(a); free(b); return -2; }
    for (int64_t k = 0; k < ext[0]; ++k)
        for (int64_t j = 0; j < ext[1]; ++j)
            for (int64_t i = 0; i < ext[2]; ++i)
                a[(k * ext[1] + j) * ext[2] + i] =
                    or_read(u0, &g, bc, lo[0] + k, lo[1] + j, lo[2] + i);
    /* A window cell whose unwrapped coordinate lies outside the grid under
     * the zero rule is a ghost: it holds 0 at every step.  After step t only
     * cells at least rad*t from the window edge are still exact, so each
     * step updates just that shrinking box. */
    for (int64_t t = 1; t <= steps; ++t) {
        const int64_t m = (int64_t)rad * t;
        int64_t b0[3], b1[3];
        for (int d = 0; d < 3; ++d) {
            const int real = d >= 3 - ndim;
            b0[d] = real ? m : 0;
            b1[d] = real ? ext[d] - m : 1;
        }
        for (int64_t k = b0[0]; k < b1[0]; ++k)
            for (int64_t j = b0[1]; j < b1[1]; ++j)
                for (int64_t i = b0[2]; i < b1[2]; ++i) {
                    const int64_t gz = lo[0] + k, gy = lo[1] + j, gx = lo[2] + i;
                    const int ghost = gz < 0 || gz >= g.n[0] || gy < 0 || gy >= g.n[1] ||
                                      gx < 0 || gx >= g.n[2];
                    double v = 0.0;
                    if (!(ghost && bc == OR_BC_ZERO)) {
                        for (int32_t p = 0; p < npoints; ++p) {
                            const int64_t kk = k + off[3 * p], jj = j + off[3 * p + 1],
                                          ii = i + off[3 * p + 2];
                            v += weights[p] * a[(kk * ext[1] + jj) * ext[2] + ii];
                        }
                    }
                    b[(k * ext[1] + j) * ext[2] + i] = v;
                }
        double* tmp = a; a = b; b = tmp;
    }
    *out = a[(h * (ndim >= 3) * ext[1] + h * (ndim >= 2)) * ext[2] + h];
    free(a);
    free(b);
    return 0;
}

/* Variable-coefficient heat step (3D, zero-Dirichlet ghost layer):
 *   u_new[i] = u[i] + alpha * sum over the 6 faces f=(axis,sign) of
 *              kappa_f * (u[i+f] - u[i]),
 *   kappa_f = (k[i] + k[i+f]) / 2 for an interior face,
 *   kappa_f = k[i] with u[i+f] = 0 for a face on the grid boundary.
 * Faces are visited axis z, y, x and sign -, + within an axis. */
static void oracle_varcoef_step(const or_grid* g, const double* k, double alpha,
                                const double* u, double* un, int nt)
{
    const int64_t nz = g->n[0], ny = g->n[1], nx = g->n[2];
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t i = (z * ny + y) * nx + x;
                int64_t c[3] = {z, y, x};
                double acc = 0.0;
                for (int d = 0; d < 3; ++d)
                    for (int sg = -1; sg <= 1; sg += 2) {
                        int64_t q[3] = {c[0], c[1], c[2]};
                        q[d] += sg;
                        if (q[d] < 0 || q[d] >= g->n[d]) {
                            acc += k[i] * (0.0 - u[i]);
                        } else {
                            const int64_t j = (q[0] * ny + q[1]) * nx + q[2];
                            acc += 0.5 * (k[i] + k[j]) * (u[j] - u[i]);
                        }
                    }
                un[i] = u[i] + alpha * acc;
            }
}

/* Forward var-coef run of `steps` steps on a 3D grid; when ckpts != NULL the
 * state u^{c*every} is copied to ckpts + c*N before step c*every, for
 * c = 0 .. ceil(steps/every)-1. */
int oracle_varcoef_forward(const int64_t* shape3, const double* k, double alpha,
                           int64_t steps, double* u, int64_t every, double* ckpts,
                           int32_t nthreads)
{
    or_grid g;
    if (or_setup(3, shape3, &g) || !k || !u || steps < 0 || (ckpts && every < 1)) return -1;
    double* other = (double*)malloc(sizeof(double) * (size_t)g.cells);
    if (!other) return -2;
    double* src = u;
    double* dst = other;
    const int nt = or_threads(nthreads);
    for (int64_t t = 0; t < steps; ++t) {
        if (ckpts && t % every == 0)
            memcpy(ckpts + (t / every) * g.cells, src, sizeof(double) * (size_t)g.cells);
        oracle_varcoef_step(&g, k, alpha, src, dst, nt);
        double* tmp = src; src = dst; dst = tmp;
    }
    if (src != u) memcpy(u, src, sizeof(double) * (size_t)g.cells);
    free(other);
    return 0;
}

/* Reverse mode of oracle_varcoef_step at state u (= u^n), given
 * lam = dL/du^{n+1}: returns lam_out = dL/du^n and adds dL/dk into gk.
 * Written as the scatter transpose of the forward loop. */
static void oracle_varcoef_step_adjoint(const or_grid* g, const double* k, double alpha,
                                        const double* u, const double* lam,
                                        double* lam_out, double* gk)
{
    const int64_t nz = g->n[0], ny = g->n[1], nx = g->n[2];
    memset(lam_out, 0, sizeof(double) * (size_t)g->cells);
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t i = (z * ny + y) * nx + x;
                const double gi = lam[i];
                int64_t c[3] = {z, y, x};
                /* d u_new[i] / d u[i] from the leading "u[i] +" */
                lam_out[i] += gi;
                for (int d = 0; d < 3; ++d)
                    for (int sg = -1; sg <= 1; sg += 2) {
                        int64_t q[3] = {c[0], c[1], c[2]};
                        q[d] += sg;
                        if (q[d] < 0 || q[d] >= g->n[d]) {
                            /* term alpha * k[i] * (0 - u[i]) */
                            lam_out[i] -= gi * alpha * k[i];
                            if (gk) gk[i] += gi * alpha * (0.0 - u[i]);
                        } else {
                            const int64_t j = (q[0] * ny + q[1]) * nx + q[2];
                            const double kap = 0.5 * (k[i] + k[j]);
                            /* term alpha * kap * (u[j] - u[i]) */
                            lam_out[j] += gi * alpha * kap;
                            lam_out[i] -= gi * alpha * kap;
                            if (gk) {
                                const double dk = gi * alpha * (u[j] - u[i]);
                                gk[i] += 0.5 * dk;
                                gk[j] += 0.5 * dk;
                            }
                        }
                    }
            }
}

/* Full adjoint of oracle_varcoef_forward: `lam` holds dL/du^T on entry and
 * dL/du^0 on exit; gk (may be NULL) receives += dL/dk.  u0 is the initial
 * state; the forward states are recomputed from it (no checkpoints needed
 * in the reference: it stores every state). */
int oracle_varcoef_adjoint(const int64_t* shape3, const double* k, double alpha,
                           int64_t steps, const double* u0, double* lam, double* gk)
{
    or_grid g;
    if (or_setup(3, shape3, &g) || !k || !u0 || !lam || steps < 0) return -1;
    const size_t N = (size_t)g.cells;
    double* states = (double*)malloc(sizeof(double) * N * (size_t)(steps > 0 ? steps : 1));
    double* tmp = (double*)malloc(sizeof(double) * N);
    if (!states || !tmp) { free(states); free(tmp); return -2; }
    if (steps > 0) memcpy(states, u0, sizeof(double) * N);
    for (int64_t t = 1; t < steps; ++t)
        oracle_varcoef_step(&g, k, alpha, states + (t - 1) * N, states + t * N, 1);
    for (int64_t t = steps - 1; t >= 0; --t) {
        oracle_varcoef_step_adjoint(&g, k, alpha, states + t * N, lam, tmp, gk);
        memcpy(lam, tmp, sizeof(double) * N);
    }
    free(states);
    free(tmp);
    return 0;
}

/* Heat carried out of the grid (zero rule only).  A step sends w[p] * u[c]
 * from cell c to cell c - off[p] (the cell that reads c through point p);
 * when that cell lies outside the grid the amount leaves the domain across
 * the zero-Dirichlet boundary.  This runs `steps` steps exactly as
 * oracle_sweep does and adds, for every step, the amount that leaves to
 * *flux (FP64).  With weights summing to 1 the total of u drops by exactly
 * the outflow in exact arithmetic; the tests use that as a pin. */
int oracle_sweep_flux(int32_t ndim, const int64_t* shape, int32_t npoints,
                      const int32_t* offsets, const double* weights, int64_t steps,
                      double* u, double* flux)
{
    or_grid g;
    if (or_setup(ndim, shape, &g) || npoints < 1 || npoints > 125 || !offsets || !weights ||
        !u || !flux || steps < 0)
        return -1;
    int32_t off[125 * 3];
    for (int32_t p = 0; p < npoints; ++p) {
        off[3 * p + 0] = off[3 * p + 1] = off[3 * p + 2] = 0;
        for (int d = 0; d < ndim; ++d) off[3 * p + 3 - ndim + d] = offsets[p * ndim + d];
    }
    double* state = (double*)malloc(sizeof(double) * (size_t)g.cells);
    if (!state) return -2;
    memcpy(state, u, sizeof(double) * (size_t)g.cells);
    double out = 0.0;
    for (int64_t t = 0; t < steps; ++t) {
        /* what this step sends outside, from the state it reads */
        for (int64_t z = 0; z < g.n[0]; ++z)
            for (int64_t y = 0; y < g.n[1]; ++y)
                for (int64_t x = 0; x < g.n[2]; ++x) {
                    const double v = state[(z * g.n[1] + y) * g.n[2] + x];
                    for (int32_t p = 0; p < npoints; ++p) {
                        const int64_t tz = z - off[3 * p], ty = y - off[3 * p + 1], tx = x - off[3 * p + 2];
                        if (tz < 0 || tz >= g.n[0] || ty < 0 || ty >= g.n[1] || tx < 0 || tx >= g.n[2])
                            out += weights[p] * v;
                    }
                }
        if (oracle_sweep(ndim, shape, npoints, offsets, weights, OR_BC_ZERO, 1, state, 1) != 0) {
            free(state);
            return -3;
        }
    }
    memcpy(u, state, sizeof(double) * (size_t)g.cells);
    free(state);
    *flux += out;
    return 0;
}
