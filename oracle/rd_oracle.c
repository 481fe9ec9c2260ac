/*
 * rd_oracle.c -- plain FP64 dense-grid CPU oracle for sparse-grid reaction-diffusion.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no code,
 * header, table or constant with the HIP library and must never be reached from
 * the product path.
 *
 * What it computes (paper: Stark & Sbalzarini, "An open-source pipeline for
 * solving continuous reaction-diffusion models in image-based geometries of
 * porous media", arXiv 2304.11165):
 *
 *  - the reaction-diffusion PDE du/dt = div(D grad u) + f(u)  (section "Methods",
 *    eq. reaction_diffusion) inside Omega = {phi > 0};
 *  - discretised by FTCS: forward Euler in time, centred second differences in
 *    space (section "Discretization and numerical methods"), written in the
 *    conservative per-axis flux form of the inhomogeneous-diffusion functor of
 *    appendix "Code examples": u' = u + dt/dx^2 * sum_axes [D+(u+ - u) - D-(u - u-)],
 *    D+- the arithmetic mean of D at the two points; D at a point is D_s * e(x) with
 *    an optional per-voxel factor e (e = 1 without one: constant D per species);
 *  - the smooth diffusivity D(phi) = D_min + D_max / (1 + exp(-(g1 + g2 phi))) of
 *    section "Level-set method ...", eq. inhomog_diffusion_coefficient, used as e;
 *  - no-flux walls by the mirror rule of the same section: a neighbour outside
 *    Omega takes the centre's value, so that face's flux is zero;
 *  - reactions evaluated at the old time level (law of mass action, first order);
 *  - a reactive wall (Robin) with flux k_R * u per wall face, the per-face form of
 *    the paper's surface-restricted sink (section "Application example 2");
 *  - or that sink in volumetric form: rate k_s * u on the voxels of a near-surface
 *    band selected by the level set (the same section);
 *  - a Dirichlet face: the active voxels of a box face plane hold a fixed value
 *    (section "Application example 1": a solute enters from one face).
 *
 * The grid is a plain dense array (nz, ny, nx), x fastest, with a uint8 mask
 * (1 = active voxel in Omega).  No blocks, no index, no fusion.  Loops are the
 * definitions written out.
 *
 * Species arrays are stacked: c[s * N + p], N = nx*ny*nz.
 * dir_face[s*6 + f] != 0 marks face f (0:-x 1:+x 2:-y 3:+y 4:-z 5:+z) of species s
 * as Dirichlet; the held value is whatever c holds there on entry.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, k) ((int64_t)(k) * ny * nx + (int64_t)(j) * nx + (int64_t)(i))

/* Is voxel (i,j,k) a fixed-value voxel of species s?  It must be active and lie
 * on the plane of a face flagged Dirichlet for s. */
static int is_dirichlet(const uint8_t *dir_face, int s, int64_t i, int64_t j, int64_t k,
                        int64_t nx, int64_t ny, int64_t nz)
{
    const uint8_t *f = dir_face ? dir_face + 6 * s : NULL;
    if (!f) return 0;
    if (f[0] && i == 0) return 1;
    if (f[1] && i == nx - 1) return 1;
    if (f[2] && j == 0) return 1;
    if (f[3] && j == ny - 1) return 1;
    if (f[4] && k == 0) return 1;
    if (f[5] && k == nz - 1) return 1;
    return 0;
}

/* The first Dirichlet face (in face order) that voxel (i,j,k) lies on for s, or -1. */
static int dirichlet_face_of(const uint8_t *dir_face, int s, int64_t i, int64_t j, int64_t k,
                             int64_t nx, int64_t ny, int64_t nz)
{
    const uint8_t *f = dir_face + 6 * s;
    if (f[0] && i == 0) return 0;
    if (f[1] && i == nx - 1) return 1;
    if (f[2] && j == 0) return 2;
    if (f[3] && j == ny - 1) return 3;
    if (f[4] && k == 0) return 4;
    if (f[5] && k == nz - 1) return 5;
    return -1;
}

/* Neighbour offsets in the order -x,+x,-y,+y,-z,+z. */
static const int DI[6] = {-1, 1, 0, 0, 0, 0};
static const int DJ[6] = {0, 0, -1, 1, 0, 0};
static const int DK[6] = {0, 0, 0, 0, -1, 1};

static int in_box(int64_t i, int64_t j, int64_t k, int64_t nx, int64_t ny, int64_t nz)
{
    return i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
}

/* Number of wall faces of voxel p: in-box face neighbours that are not active.
 * Box faces are not walls. */
static int wall_count(const uint8_t *active, int64_t i, int64_t j, int64_t k,
                      int64_t nx, int64_t ny, int64_t nz)
{
    int n = 0;
    for (int f = 0; f < 6; ++f) {
        int64_t a = i + DI[f], b = j + DJ[f], c = k + DK[f];
        if (in_box(a, b, c, nx, ny, nz) && !active[IDX(a, b, c)]) ++n;
    }
    return n;
}

/*
 * One FTCS step for every species: cout = step(cin).
 *  D[s]        diffusion coefficient of species s
 *  robin_k[s]  wall-uptake coefficient k_R of species s (0: plain no-flux); may be NULL
 *  reactions   r_from[r] -> r_to[r] (r_to = -1: decay) with first-order rate r_rate[r]
 *  source      optional volumetric source nspec*N (added as dt*source), may be NULL
 *  eps         optional per-voxel diffusivity factor (N values): D at voxel p is
 *              D[s] * eps[p]; NULL means eps = 1
 *  sink_k      optional volumetric sink rate per species, applied (as -dt*k_s*u) on the
 *  sink_mask   voxels with sink_mask[p] != 0; either NULL: no sink
 */
static void ftcs_step(int64_t nx, int64_t ny, int64_t nz, double dx, const uint8_t *active,
                      int nspec, const double *D, const double *robin_k, const uint8_t *dir_face,
                      int nreact, const int32_t *r_from, const int32_t *r_to, const double *r_rate,
                      const double *source, const double *eps, const double *sink_k,
                      const uint8_t *sink_mask, double dt, const double *cin, double *cout)
{
    const int64_t N = nx * ny * nz;
    for (int s = 0; s < nspec; ++s) {
        const double *u = cin + (int64_t)s * N;
        double *uo = cout + (int64_t)s * N;
        const double kR = robin_k ? robin_k[s] : 0.0;
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nz; ++k) {
            for (int64_t j = 0; j < ny; ++j) {
                for (int64_t i = 0; i < nx; ++i) {
                    const int64_t p = IDX(i, j, k);
                    if (!active[p]) { uo[p] = 0.0; continue; }
                    if (is_dirichlet(dir_face, s, i, j, k, nx, ny, nz)) { uo[p] = u[p]; continue; }
                    const double uc = u[p];
                    const double Dc = D[s] * (eps ? eps[p] : 1.0);
                    /* neighbour values and coefficients with the mirror rule: outside
                     * Omega (or the box) both take the centre's, u -> u_c, D -> D_c */
                    double nb[6], Dn[6];
                    int nwall = 0;
                    for (int f = 0; f < 6; ++f) {
                        int64_t a = i + DI[f], b = j + DJ[f], c = k + DK[f];
                        nb[f] = uc;
                        Dn[f] = Dc;
                        if (!in_box(a, b, c, nx, ny, nz)) continue;
                        int64_t q = IDX(a, b, c);
                        if (active[q]) {
                            nb[f] = u[q];
                            Dn[f] = D[s] * (eps ? eps[q] : 1.0);
                        } else {
                            ++nwall;
                        }
                    }
                    /* arithmetic-mean D at the half points */
                    double Dh[6];
                    for (int f = 0; f < 6; ++f) Dh[f] = 0.5 * (Dc + Dn[f]);
                    double flux = Dh[1] * (nb[1] - uc) - Dh[0] * (uc - nb[0])   /* x */
                                + Dh[3] * (nb[3] - uc) - Dh[2] * (uc - nb[2])   /* y */
                                + Dh[5] * (nb[5] - uc) - Dh[4] * (uc - nb[4]);  /* z */
                    double un = uc + dt * (1.0 / (dx * dx)) * flux;
                    /* reactive wall: flux k_R*u through each wall face of area dx^2 */
                    un -= dt * kR * (double)nwall * uc / dx;
                    /* volumetric near-surface sink */
                    if (sink_k && sink_mask && sink_mask[p]) un -= dt * sink_k[s] * uc;
                    /* first-order reactions at the old time level */
                    for (int r = 0; r < nreact; ++r) {
                        double rate = r_rate[r] * cin[(int64_t)r_from[r] * N + p];
                        if (r_from[r] == s) un -= dt * rate;
                        if (r_to[r] == s) un += dt * rate;
                    }
                    if (source) un += dt * source[(int64_t)s * N + p];
                    uo[p] = un;
                }
            }
        }
    }
}

/* Run nsteps FTCS steps in place on c (nspec*N).  work: nspec*N scratch (may be NULL).
 * eps: per-voxel diffusivity factor (N values) or NULL. */
int orc_ftcs_run_ext(int64_t nx, int64_t ny, int64_t nz, double dx, const uint8_t *active,
                     int nspec, const double *D, const double *robin_k, const uint8_t *dir_face,
                     int nreact, const int32_t *r_from, const int32_t *r_to, const double *r_rate,
                     const double *source, const double *eps, const double *sink_k,
                     const uint8_t *sink_mask, double dt, int64_t nsteps, double *c, double *work)
{
    const int64_t N = nx * ny * nz;
    double *tmp = work;
    int own = 0;
    if (!tmp) {
        tmp = (double *)malloc(sizeof(double) * (size_t)(N * nspec));
        if (!tmp) return 1;
        own = 1;
    }
    double *a = c, *b = tmp;
    for (int64_t n = 0; n < nsteps; ++n) {
        ftcs_step(nx, ny, nz, dx, active, nspec, D, robin_k, dir_face, nreact, r_from, r_to,
                  r_rate, source, eps, sink_k, sink_mask, dt, a, b);
        double *t = a; a = b; b = t;
    }
    if (a != c) memcpy(c, a, sizeof(double) * (size_t)(N * nspec));
    if (own) free(tmp);
    return 0;
}

int orc_ftcs_run(int64_t nx, int64_t ny, int64_t nz, double dx, const uint8_t *active,
                 int nspec, const double *D, const double *robin_k, const uint8_t *dir_face,
                 int nreact, const int32_t *r_from, const int32_t *r_to, const double *r_rate,
                 const double *source, double dt, int64_t nsteps, double *c, double *work)
{
    return orc_ftcs_run_ext(nx, ny, nz, dx, active, nspec, D, robin_k, dir_face, nreact, r_from,
                            r_to, r_rate, source, NULL, NULL, NULL, dt, nsteps, c, work);
}

/* Smooth diffusivity of eq. inhomog_diffusion_coefficient (section "Level-set method
 * for image-based geometry reconstruction"): out[i] = d_min + d_max / (1 +
 * exp(-(g1 + g2 * phi[i]))), FP64. */
void orc_smooth_diffusivity(int64_t n, const double *phi, double d_min, double d_max, double g1,
                            double g2, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = d_min + d_max / (1.0 + exp(-(g1 + g2 * phi[i])));
}

/*
 * Balance terms of species s for the field c (nspec*N):
 *   mass          sum over free voxels of c * dx^3       (paper: total-mass monitor)
 *   inflow[6]     per Dirichlet face f: sum over (q Dirichlet on f, p free active
 *                 neighbour of q) of D_h*(c_q - c_p)*dx, D_h the mean of D at q and p
 *   robin         sum over free voxels of k_R * n_wall * c * dx^2 (+ k_s * c * dx^3 on the
 *                 sink band)
 *   react         sum over free voxels of the reaction rate of s, times dx^3
 * A voxel is "free" for s if it is active and not a Dirichlet voxel of s.  With
 * these terms one FTCS step satisfies M' - M = dt*(sum(inflow) - robin + react).
 */
int orc_balance_ext(int64_t nx, int64_t ny, int64_t nz, double dx, const uint8_t *active,
                    int nspec, const double *D, const double *robin_k, const uint8_t *dir_face,
                    int nreact, const int32_t *r_from, const int32_t *r_to, const double *r_rate,
                    const double *eps, const double *sink_k, const uint8_t *sink_mask,
                    const double *c, int s, double *mass, double *inflow, double *robin,
                    double *react)
{
    const int64_t N = nx * ny * nz;
    const double *u = c + (int64_t)s * N;
    const double kR = robin_k ? robin_k[s] : 0.0;
    (void)nspec;
    /* per-plane partial sums (9 per plane: mass, robin, react, inflow[6]), added in
     * plane order afterwards, so the result does not depend on the thread count */
    double *part = (double *)calloc((size_t)nz * 9, sizeof(double));
    if (!part) return 1;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k) {
        double m = 0.0, rb = 0.0, re = 0.0;
        double fl[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t p = IDX(i, j, k);
                if (!active[p]) continue;
                int df = dir_face ? dirichlet_face_of(dir_face, s, i, j, k, nx, ny, nz) : -1;
                if (df >= 0) {
                    for (int f = 0; f < 6; ++f) {
                        int64_t a = i + DI[f], b = j + DJ[f], cc = k + DK[f];
                        if (!in_box(a, b, cc, nx, ny, nz)) continue;
                        int64_t q = IDX(a, b, cc);
                        if (!active[q]) continue;
                        if (is_dirichlet(dir_face, s, a, b, cc, nx, ny, nz)) continue;
                        /* arithmetic mean of D at the two voxels, as in the step */
                        const double Dh = 0.5 * (D[s] * (eps ? eps[p] : 1.0) +
                                                 D[s] * (eps ? eps[q] : 1.0));
                        fl[df] += Dh * (u[p] - u[q]) * dx;
                    }
                    continue;
                }
                m += u[p] * dx * dx * dx;
                rb += kR * (double)wall_count(active, i, j, k, nx, ny, nz) * u[p] * dx * dx;
                if (sink_k && sink_mask && sink_mask[p]) rb += sink_k[s] * u[p] * dx * dx * dx;
                for (int r = 0; r < nreact; ++r) {
                    double rate = r_rate[r] * c[(int64_t)r_from[r] * N + p];
                    if (r_from[r] == s) re -= rate * dx * dx * dx;
                    if (r_to[r] == s) re += rate * dx * dx * dx;
                }
            }
        double *pk = part + 9 * k;
        pk[0] = m;
        pk[1] = rb;
        pk[2] = re;
        for (int f = 0; f < 6; ++f) pk[3 + f] = fl[f];
    }
    double m = 0.0, rb = 0.0, re = 0.0;
    double fl[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t k = 0; k < nz; ++k) {
        m += part[9 * k];
        rb += part[9 * k + 1];
        re += part[9 * k + 2];
        for (int f = 0; f < 6; ++f) fl[f] += part[9 * k + 3 + f];
    }
    free(part);
    *mass = m;
    *robin = rb;
    *react = re;
    for (int f = 0; f < 6; ++f) inflow[f] = fl[f];
    return 0;
}

int orc_balance(int64_t nx, int64_t ny, int64_t nz, double dx, const uint8_t *active,
                int nspec, const double *D, const double *robin_k, const uint8_t *dir_face,
                int nreact, const int32_t *r_from, const int32_t *r_to, const double *r_rate,
                const double *c, int s, double *mass, double *inflow, double *robin, double *react)
{
    return orc_balance_ext(nx, ny, nz, dx, active, nspec, D, robin_k, dir_face, nreact, r_from,
                           r_to, r_rate, NULL, NULL, NULL, c, s, mass, inflow, robin, react);
}

/* Diffusive flux of one species through the plane between index i and i+1 along
 * `axis` (0=x,1=y,2=z), counted positive in the +axis direction:
 * sum over pairs of active voxels straddling the plane of D*(u_i - u_{i+1})*dx. */
double orc_plane_flux(int64_t nx, int64_t ny, int64_t nz, double dx, const uint8_t *active,
                      double D, const double *u, int axis, int64_t i0)
{
    double q = 0.0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t c0 = axis == 0 ? i : axis == 1 ? j : k;
                if (c0 != i0) continue;
                int64_t a = i + (axis == 0), b = j + (axis == 1), cc = k + (axis == 2);
                if (!in_box(a, b, cc, nx, ny, nz)) continue;
                int64_t p = IDX(i, j, k), r = IDX(a, b, cc);
                if (active[p] && active[r]) q += D * (u[p] - u[r]) * dx;
            }
    return q;
}

/* The same flux with a per-voxel diffusivity factor: each straddling pair carries
 * D * (eps_i + eps_{i+1}) / 2 * (u_i - u_{i+1}) * dx (the face coefficient of the step). */
double orc_plane_flux_eps(int64_t nx, int64_t ny, int64_t nz, double dx, const uint8_t *active,
                          double D, const double *eps, const double *u, int axis, int64_t i0)
{
    double q = 0.0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t c0 = axis == 0 ? i : axis == 1 ? j : k;
                if (c0 != i0) continue;
                int64_t a = i + (axis == 0), b = j + (axis == 1), cc = k + (axis == 2);
                if (!in_box(a, b, cc, nx, ny, nz)) continue;
                int64_t p = IDX(i, j, k), r = IDX(a, b, cc);
                if (active[p] && active[r]) q += D * 0.5 * (eps[p] + eps[r]) * (u[p] - u[r]) * dx;
            }
    return q;
}

/* ---------------------------------------------------------------------------
 * Steady state of pure diffusion (no reactions, no Robin) with the Dirichlet data
 * held in u: the discrete Laplace problem on the free voxels,
 *     (A u)_p = sum over active neighbours q of (u_p - u_q) = 0   for free p.
 * Written as A_ff u_f = b with b_p = sum of Dirichlet neighbour values.
 * free[p] = 1 for free voxels (active, not Dirichlet).
 * ------------------------------------------------------------------------- */

/* r = b - A_ff u_f on free voxels (0 elsewhere); returns ||r||^2, and ||b||^2 in *bb. */
static double steady_residual(int64_t nx, int64_t ny, int64_t nz, const uint8_t *active,
                              const uint8_t *free_, const double *u, double *r, double *bb)
{
    /* per-plane partials, added in plane order (independent of the thread count) */
    double *part = (double *)calloc((size_t)nz * 2, sizeof(double));
    if (!part) return NAN;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k) {
        double rr = 0.0, b2 = 0.0;
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t p = IDX(i, j, k);
                if (!free_[p]) { if (r) r[p] = 0.0; continue; }
                double bp = 0.0, au = 0.0;
                for (int f = 0; f < 6; ++f) {
                    int64_t a = i + DI[f], b = j + DJ[f], c = k + DK[f];
                    if (!in_box(a, b, c, nx, ny, nz)) continue;
                    int64_t q = IDX(a, b, c);
                    if (!active[q]) continue;
                    au += u[p];
                    if (free_[q]) au -= u[q];
                    else bp += u[q];
                }
                double rp = bp - au;
                if (r) r[p] = rp;
                rr += rp * rp;
                b2 += bp * bp;
            }
        part[2 * k] = rr;
        part[2 * k + 1] = b2;
    }
    double rr = 0.0, b2 = 0.0;
    for (int64_t k = 0; k < nz; ++k) {
        rr += part[2 * k];
        b2 += part[2 * k + 1];
    }
    free(part);
    if (bb) *bb = b2;
    return rr;
}

/* Jacobi iteration u_p <- (b_p + sum_free_nb u_q) / n_active_nb(p) until
 * ||r||/||b|| <= tol.  Voxels with no active neighbour keep their value. */
int orc_steady_jacobi(int64_t nx, int64_t ny, int64_t nz, const uint8_t *active,
                      const uint8_t *free_, double *u, double tol, int64_t max_iters,
                      int64_t check_every, int64_t *iters, double *rel_res)
{
    const int64_t N = nx * ny * nz;
    double *v = (double *)malloc(sizeof(double) * (size_t)N);
    if (!v) return 1;
    memcpy(v, u, sizeof(double) * (size_t)N);
    double bb = 0.0, rr = steady_residual(nx, ny, nz, active, free_, u, NULL, &bb);
    double rel = bb > 0 ? sqrt(rr / bb) : 0.0;
    int64_t it = 0;
    while (rel > tol && it < max_iters) {
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    int64_t p = IDX(i, j, k);
                    if (!free_[p]) { v[p] = u[p]; continue; }
                    double s = 0.0;
                    int n = 0;
                    for (int f = 0; f < 6; ++f) {
                        int64_t a = i + DI[f], b = j + DJ[f], c = k + DK[f];
                        if (!in_box(a, b, c, nx, ny, nz)) continue;
                        int64_t q = IDX(a, b, c);
                        if (!active[q]) continue;
                        s += u[q];
                        ++n;
                    }
                    v[p] = n ? s / (double)n : u[p];
                }
        memcpy(u, v, sizeof(double) * (size_t)N);
        ++it;
        if (it % check_every == 0 || it == max_iters) {
            rr = steady_residual(nx, ny, nz, active, free_, u, NULL, &bb);
            rel = bb > 0 ? sqrt(rr / bb) : 0.0;
        }
    }
    free(v);
    *iters = it;
    *rel_res = rel;
    return rel <= tol ? 0 : 2;
}

/* Conjugate gradients on A_ff u_f = b (A_ff is symmetric positive semi-definite;
 * components without Dirichlet contact have b = 0 there and stay at the initial
 * guess's value if that is 0).  u holds the Dirichlet data and the initial guess. */
int orc_steady_cg(int64_t nx, int64_t ny, int64_t nz, const uint8_t *active,
                  const uint8_t *free_, double *u, double tol, int64_t max_iters,
                  int64_t *iters, double *rel_res)
{
    const int64_t N = nx * ny * nz;
    double *r = (double *)calloc((size_t)N, sizeof(double));
    double *p = (double *)calloc((size_t)N, sizeof(double));
    double *ap = (double *)calloc((size_t)N, sizeof(double));
    if (!r || !p || !ap) { free(r); free(p); free(ap); return 1; }
    double bb = 0.0;
    double rr = steady_residual(nx, ny, nz, active, free_, u, r, &bb);
    memcpy(p, r, sizeof(double) * (size_t)N);
    int64_t it = 0;
    double rel = bb > 0 ? sqrt(rr / bb) : 0.0;
    const int64_t NP = nx * ny; /* voxels per z-plane */
    double *part = (double *)calloc((size_t)nz, sizeof(double));
    if (!part) { free(r); free(p); free(ap); return 1; }
    while (rel > tol && it < max_iters) {
        /* ap = A_ff p (p is zero off the free set); p.ap as per-plane partials added
         * in plane order */
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nz; ++k) {
            double pap_k = 0.0;
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    int64_t q0 = IDX(i, j, k);
                    if (!free_[q0]) { ap[q0] = 0.0; continue; }
                    double s = 0.0;
                    for (int f = 0; f < 6; ++f) {
                        int64_t a = i + DI[f], b = j + DJ[f], c = k + DK[f];
                        if (!in_box(a, b, c, nx, ny, nz)) continue;
                        int64_t q = IDX(a, b, c);
                        if (!active[q]) continue;
                        s += p[q0];
                        if (free_[q]) s -= p[q];
                    }
                    ap[q0] = s;
                    pap_k += p[q0] * s;
                }
            part[k] = pap_k;
        }
        double pap = 0.0;
        for (int64_t k = 0; k < nz; ++k) pap += part[k];
        if (pap <= 0.0) break;
        double alpha = rr / pap;
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nz; ++k) {
            double rr_k = 0.0;
            for (int64_t q = k * NP; q < (k + 1) * NP; ++q) {
                if (!free_[q]) continue;
                u[q] += alpha * p[q];
                r[q] -= alpha * ap[q];
                rr_k += r[q] * r[q];
            }
            part[k] = rr_k;
        }
        double rr_new = 0.0;
        for (int64_t k = 0; k < nz; ++k) rr_new += part[k];
        double beta = rr_new / rr;
        rr = rr_new;
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < N; ++q)
            p[q] = free_[q] ? r[q] + beta * p[q] : 0.0;
        ++it;
        rel = bb > 0 ? sqrt(rr / bb) : 0.0;
    }
    free(part);
    /* report the true residual, not the recursively updated one */
    rr = steady_residual(nx, ny, nz, active, free_, u, NULL, &bb);
    rel = bb > 0 ? sqrt(rr / bb) : 0.0;
    free(r); free(p); free(ap);
    *iters = it;
    *rel_res = rel;
    return rel <= tol ? 0 : 2;
}

/* ---------------------------------------------------------------------------
 * Discrete adjoint of single-species diffusion-decay FTCS with Dirichlet faces:
 *     c^{n+1}_p = c^n_p + a * sum_{q active nb}(c^n_q - c^n_p) - b * c^n_p   (free p)
 *     a = D dt / dx^2,  b = k dt;  Dirichlet and inactive voxels do not change.
 * Loss L = 1/2 sum_free (c^N - c*)^2.  With lambda^N = c^N - c* on free voxels,
 *     lambda^n = (dc^{n+1}/dc^n)^T lambda^{n+1}  (restricted to free voxels),
 *     dL/dD = sum_n <lambda^{n+1}, dt/dx^2 * sum_{q}(c^n_q - c^n_p)>,
 *     dL/dk = sum_n <lambda^{n+1}, -dt * c^n>.
 * The transpose is written out entry by entry: for free q,
 *     lambda^n_q = (1 - a*nact(q) - b) lambda^{n+1}_q + a * sum_{p free nb of q} lambda^{n+1}_p.
 * States are re-computed from checkpoints stored every `stride` steps.
 * ------------------------------------------------------------------------- */
int orc_adjoint_decay(int64_t nx, int64_t ny, int64_t nz, double dx, const uint8_t *active,
                      const uint8_t *dir_face /* 6 */, double D, double k, double dt,
                      int64_t nsteps, int64_t stride, const double *c0, const double *target,
                      double *loss, double *dL_dD, double *dL_dk, double *cN)
{
    const int64_t N = nx * ny * nz;
    if (stride < 1) stride = 1;
    const int64_t ncp = (nsteps + stride - 1) / stride + 1;
    double *cps = (double *)malloc(sizeof(double) * (size_t)(N * ncp));
    double *seg = (double *)malloc(sizeof(double) * (size_t)(N * (stride + 1)));
    double *lam = (double *)calloc((size_t)N, sizeof(double));
    double *lam2 = (double *)calloc((size_t)N, sizeof(double));
    double *cur = (double *)malloc(sizeof(double) * (size_t)N);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)N);
    uint8_t *free_ = (uint8_t *)malloc((size_t)N);
    int32_t rf = 0, rt = -1;
    if (!cps || !seg || !lam || !lam2 || !cur || !tmp || !free_) {
        free(cps); free(seg); free(lam); free(lam2); free(cur); free(tmp); free(free_);
        return 1;
    }
    for (int64_t kk = 0; kk < nz; ++kk)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t p = IDX(i, j, kk);
                free_[p] = active[p] && !is_dirichlet(dir_face, 0, i, j, kk, nx, ny, nz);
            }
    /* forward sweep with checkpoints */
    memcpy(cur, c0, sizeof(double) * (size_t)N);
    memcpy(cps, cur, sizeof(double) * (size_t)N);
    for (int64_t n = 0; n < nsteps; ++n) {
        ftcs_step(nx, ny, nz, dx, active, 1, &D, NULL, dir_face, 1, &rf, &rt, &k, NULL, NULL, NULL, NULL, dt, cur, tmp);
        memcpy(cur, tmp, sizeof(double) * (size_t)N);
        if ((n + 1) % stride == 0)
            memcpy(cps + ((n + 1) / stride) * N, cur, sizeof(double) * (size_t)N);
    }
    if (cN) memcpy(cN, cur, sizeof(double) * (size_t)N);
    double L = 0.0;
    for (int64_t p = 0; p < N; ++p) {
        if (!free_[p]) { lam[p] = 0.0; continue; }
        double d = cur[p] - target[p];
        L += 0.5 * d * d;
        lam[p] = d;
    }
    const double a = D * dt / (dx * dx), b = k * dt;
    double gD = 0.0, gk = 0.0;
    double *gpart = (double *)calloc((size_t)nz * 2, sizeof(double));
    if (!gpart) {
        free(cps); free(seg); free(lam); free(lam2); free(cur); free(tmp); free(free_);
        return 1;
    }
    /* backward over segments [s0, s1) */
    for (int64_t s1 = nsteps; s1 > 0;) {
        int64_t s0 = ((s1 - 1) / stride) * stride;
        int64_t len = s1 - s0;
        memcpy(seg, cps + (s0 / stride) * N, sizeof(double) * (size_t)N);
        for (int64_t m = 0; m < len - 1; ++m)
            ftcs_step(nx, ny, nz, dx, active, 1, &D, NULL, dir_face, 1, &rf, &rt, &k, NULL, NULL, NULL, NULL, dt,
                      seg + m * N, seg + (m + 1) * N);
        for (int64_t m = len - 1; m >= 0; --m) {
            const double *c = seg + m * N; /* c^{s0+m}; lam holds lambda^{s0+m+1} */
            /* gradient terms as per-plane partials, added in plane order */
#pragma omp parallel for schedule(static)
            for (int64_t kk = 0; kk < nz; ++kk) {
                double gD_k = 0.0, gk_k = 0.0;
                for (int64_t j = 0; j < ny; ++j)
                    for (int64_t i = 0; i < nx; ++i) {
                        int64_t p = IDX(i, j, kk);
                        if (!free_[p]) { lam2[p] = 0.0; continue; }
                        double lap = 0.0, lsum = 0.0;
                        int nact = 0;
                        for (int f = 0; f < 6; ++f) {
                            int64_t aa = i + DI[f], bb = j + DJ[f], cc = kk + DK[f];
                            if (!in_box(aa, bb, cc, nx, ny, nz)) continue;
                            int64_t q = IDX(aa, bb, cc);
                            if (!active[q]) continue;
                            ++nact;
                            lap += c[q] - c[p];
                            if (free_[q]) lsum += lam[q];
                        }
                        gD_k += lam[p] * dt / (dx * dx) * lap;
                        gk_k += lam[p] * (-dt) * c[p];
                        lam2[p] = (1.0 - a * (double)nact - b) * lam[p] + a * lsum;
                    }
                gpart[2 * kk] = gD_k;
                gpart[2 * kk + 1] = gk_k;
            }
            for (int64_t kk = 0; kk < nz; ++kk) {
                gD += gpart[2 * kk];
                gk += gpart[2 * kk + 1];
            }
            double *t = lam; lam = lam2; lam2 = t;
        }
        s1 = s0;
    }
    *loss = L;
    *dL_dD = gD;
    *dL_dk = gk;
    free(gpart);
    free(cps); free(seg); free(lam); free(lam2); free(cur); free(tmp); free(free_);
    return 0;
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
