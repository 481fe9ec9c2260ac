// frap.cpp -- simulated FRAP (fluorescence recovery after photobleaching) and the fit of
// an effective diffusion coefficient, paper section "Calculation of effective
// diffusion coefficient and tortuosity": the mass inside a bleached box is recorded
// while the field recovers; a free-space (all-active) box of the same size gives the
// reference recovery, and D_eff is the free-space coefficient whose recovery matches
// the porous one in the least-squares sense; tau_d = D / D_eff (eq. tortuosity).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <string>
#include <vector>

#include "rd_frap.h"
#include "rd_host.h"
#include "rd_sim.h"

static rd_status region_mass(rd_sim *sim, int species, const int32_t reg[6], double *mass)
{
    const rd_geometry &G = *sim->g;
    const int nb = (int)G.nb();
    char *ws = sim->ws;
    const SimLayout &L = sim->L;
    double *part = (double *)(ws + L.part);
    double *res = (double *)(ws + L.res) + 40;
    LAUNCHCHK(rd_launch_region_mass((int)sim->storage, G.B, (const BlockInfo *)(ws + L.info),
                                    (const uint8_t *)(ws + L.code), sim->cbase_ptr(),
                                    (const uint64_t *)(ws + L.mask), sim->field_ptr(sim->cur, species), nb, reg,
                                    part, sim->stream));
    LAUNCHCHK(rd_launch_finish_reduce(part, rd_region_rows(G.B, nb), 1, (double *)(ws + L.mid), res,
                                      sim->stream));
    HIPCHK(hipMemcpyAsync(sim->host_res, res, sizeof(double), hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(hipStreamSynchronize(sim->stream));
    const double v = sim->host_res[0];
    if (!std::isfinite(v)) return rd_fail(RD_ERR_NONFINITE, "the region holds a NaN or infinity");
    *mass = v * G.dx * G.dx * G.dx;
    return RD_OK;
}

static rd_status check_region(const rd_sim *sim, int species, const int64_t region[6], int32_t reg[6])
{
    if (!sim->ws) return rd_fail(RD_ERR_STATE, "bind a workspace first");
    if (species < 0 || species >= sim->S) return rd_fail(RD_ERR_ARG, "bad species");
    if (!region) return rd_fail(RD_ERR_ARG, "region is NULL");
    const rd_geometry &G = *sim->g;
    const int64_t n[3] = {G.nx, G.ny, G.nz};
    for (int d = 0; d < 3; ++d) {
        if (!(0 <= region[2 * d] && region[2 * d] < region[2 * d + 1] && region[2 * d + 1] <= n[d]))
            return rd_fail(RD_ERR_ARG, "region needs 0 <= lo < hi <= n on every axis");
        reg[2 * d] = (int32_t)region[2 * d];
        reg[2 * d + 1] = (int32_t)region[2 * d + 1];
    }
    return RD_OK;
}

extern "C" rd_status rd_sim_region_mass(rd_sim *sim, int species, const int64_t region[6], double *mass)
{
    if (sim && sim->g->nparts() > 1)
        return rd_fail(RD_ERR_STATE, "rd_sim_region_mass: one geometry per simulation only");
    if (!sim || !mass) return rd_fail(RD_ERR_ARG, "NULL argument");
    int32_t reg[6];
    rd_status st = check_region(sim, species, region, reg);
    if (st != RD_OK) return st;
    return region_mass(sim, species, reg, mass);
}

extern "C" rd_status rd_sim_frap_curve(rd_sim *sim, int species, const int64_t region[6], double dt,
                                       int64_t steps_per_sample, int64_t n_samples, double *curve)
{
    if (sim && sim->g->nparts() > 1)
        return rd_fail(RD_ERR_STATE, "rd_sim_frap_curve: one geometry per simulation only");
    if (!sim || !curve) return rd_fail(RD_ERR_ARG, "NULL argument");
    int32_t reg[6];
    rd_status st = check_region(sim, species, region, reg);
    if (st != RD_OK) return st;
    if (steps_per_sample < 1 || n_samples < 0) return rd_fail(RD_ERR_ARG, "need steps_per_sample >= 1, n_samples >= 0");
    st = sim->check_dt(dt);
    if (st != RD_OK) return st;
    for (int64_t k = 0; k <= n_samples; ++k) {
        if (k > 0) {
            st = sim->step(dt, steps_per_sample);
            if (st != RD_OK) return st;
        }
        st = region_mass(sim, species, reg, &curve[k]);
        if (st != RD_OK) return st;
    }
    return RD_OK;
}

// Free-space recovery at time t for coefficient D: g sampled at s_j = j ds for D_ref,
// and the diffusion equation depends on D t only, so g_D(t) = g_ref(t D / D_ref)
// (linear interpolation).
static double model(const double *g, int64_t m, double ds, double s)
{
    const double x = s / ds;
    int64_t j = (int64_t)floor(x);
    if (j >= m - 1) return g[m - 1];
    if (j < 0) return g[0];
    const double w = x - (double)j;
    return g[j] + w * (g[j + 1] - g[j]);
}

static double sq_error(int64_t n, const double *t, const double *f, int64_t m, double ds, const double *g,
                       double scale)
{
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double d = f[i] - model(g, m, ds, t[i] * scale);
        e += d * d;
    }
    return e;
}

extern "C" rd_status rd_frap_fit(int64_t n, const double *t, const double *f, int64_t m, double ds,
                                 const double *g, double D_ref, double *D_eff, double *rms)
{
    if (!t || !f || !g || !D_eff) return rd_fail(RD_ERR_ARG, "NULL argument");
    if (n < 2 || m < 2 || !(ds > 0.0) || !(D_ref > 0.0)) return rd_fail(RD_ERR_ARG, "need n, m >= 2, ds > 0, D_ref > 0");
    double tmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!(t[i] >= 0.0) || !std::isfinite(f[i])) return rd_fail(RD_ERR_ARG, "times must be >= 0, values finite");
        tmax = std::max(tmax, t[i]);
    }
    for (int64_t j = 0; j < m; ++j)
        if (!std::isfinite(g[j])) return rd_fail(RD_ERR_ARG, "reference values must be finite");
    if (!(tmax > 0.0)) return rd_fail(RD_ERR_ARG, "need a sample at t > 0");
    // scale = D / D_ref; the reference must cover t * scale, so scale <= s_max / t_max
    const double hi = (double)(m - 1) * ds / tmax;
    const double lo = hi * 1e-4;
    // coarse scan on a log grid, then golden-section search around the best point
    const int K = 400;
    int best = 0;
    double ebest = INFINITY;
    for (int k = 0; k <= K; ++k) {
        const double sc = lo * pow(hi / lo, (double)k / K);
        const double e = sq_error(n, t, f, m, ds, g, sc);
        if (e < ebest) {
            ebest = e;
            best = k;
        }
    }
    double a = log(lo) + log(hi / lo) * (double)std::max(best - 1, 0) / K;
    double b = log(lo) + log(hi / lo) * (double)std::min(best + 1, K) / K;
    const double phi = 0.5 * (sqrt(5.0) - 1.0);
    double x1 = b - phi * (b - a), x2 = a + phi * (b - a);
    double e1 = sq_error(n, t, f, m, ds, g, exp(x1)), e2 = sq_error(n, t, f, m, ds, g, exp(x2));
    for (int it = 0; it < 200 && b - a > 1e-13; ++it) {
        if (e1 <= e2) {
            b = x2; x2 = x1; e2 = e1;
            x1 = b - phi * (b - a);
            e1 = sq_error(n, t, f, m, ds, g, exp(x1));
        } else {
            a = x1; x1 = x2; e1 = e2;
            x2 = a + phi * (b - a);
            e2 = sq_error(n, t, f, m, ds, g, exp(x2));
        }
    }
    const double sc = exp(0.5 * (a + b));
    *D_eff = sc * D_ref;
    if (rms) *rms = sqrt(sq_error(n, t, f, m, ds, g, sc) / (double)n);
    return RD_OK;
}
