// rd_solve.cpp -- steady state and tortuosity by conjugate gradients (one geometry
// or a batch), and the adjoint driver.
//
// Tortuosity (eq. tortuosity: tau = D_f / D_eff) is measured from the steady
// diffusive flux Q through a box with a unit concentration drop between two
// opposite face planes: D_eff = Q L / (psi A dT), so tau = psi D dT A / (Q L), with
// psi the active volume fraction, A the box cross-section and L = (n-1) dx the
// distance between the Dirichlet planes.  A straight channel gives tau = 1.
#include <stdexcept>
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <limits>
#include <new>
#include <vector>

#include "rd_adjoint.h"
#include "rd_diff.h"
#include "rd_host.h"
#include "rd_sim.h"
#include "rd_solve.h"

namespace {

struct GeomMeta {
    int64_t nx, ny, nz;
    double psi;  // active fraction
    double dx;
    bool percolates;
};

inline double m_active(const GeomMeta &m) { return m.psi * (double)m.nx * (double)m.ny * (double)m.nz; }

struct CgOut {
    double tau = 0, rel = 0, qin = 0, qout = 0;
    int64_t iters = 0;
    bool converged = false;
};

constexpr int CHECK_EVERY = 25;  // iterations between true-residual checks (single geometry)
// stop after this many iterations (40 checks of 25) without a 10% gain of the best
// residual: CG's residual is not monotone and plateaus for hundreds of iterations on
// large volumes
constexpr int STALL_ITERS = 1000;

// Initial guess on the GPU (cg_launch_initial_guess).  Its scratch lives in solver
// vectors that CG has not used yet: the parent array in the Ap and second-p buffers,
// which are adjacent in every workspace layout (together at least 4 bytes per slot:
// `pair_bytes` from the start of Ap to the end of the second p), the cluster flags in
// r (`r_bytes`, at least 2 bytes per slot, rounded up to 256), the per-geometry
// percolation flags in the scalar area.
rd_status gpu_initial_guess(const CgArgs &a, int storage, int B, int axis, int64_t nslots, size_t pair_bytes,
                            size_t r_bytes, hipStream_t st, std::vector<char> &perc)
{
    perc.assign((size_t)a.ngeom, 0);
    if (nslots <= 0) return RD_OK;
    if (nslots >= (int64_t)UINT32_MAX) return rd_fail(RD_ERR_SHAPE, "too many slots to label");
    if (pair_bytes < 4 * (size_t)nslots || r_bytes < 2 * (size_t)nslots || r_bytes % 4 != 0)
        return rd_fail(RD_ERR_WORKSPACE, "solver vectors too small for the labelling scratch");
    uint32_t *par = (uint32_t *)a.ap;
    uint8_t *flags = (uint8_t *)a.r;
    uint32_t *pc = (uint32_t *)a.scal;
    LAUNCHCHK(rd_launch_fill_u32(flags, 0u, (int64_t)((2 * (size_t)nslots + 3) / 4), st));
    LAUNCHCHK(rd_launch_fill_u32(pc, 0u, a.ngeom, st));
    LAUNCHCHK(cg_launch_initial_guess(storage, B, a, axis, nslots, par, flags, pc, st));
    std::vector<uint32_t> h((size_t)a.ngeom);
    HIPCHK(hipMemcpyAsync(h.data(), pc, sizeof(uint32_t) * h.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int g = 0; g < a.ngeom; ++g) perc[(size_t)g] = h[(size_t)g] != 0u ? 1 : 0;
    return RD_OK;
}

rd_status copy_scal(const CgArgs &a, std::vector<double> &hs, hipStream_t st)
{
    hs.resize((size_t)a.ngeom * CG_NSCAL);
    HIPCHK(hipMemcpyAsync(hs.data(), a.scal, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return RD_OK;
}

rd_status push_scal(const CgArgs &a, const std::vector<double> &hs, hipStream_t st)
{
    HIPCHK(hipMemcpyAsync(a.scal, hs.data(), sizeof(double) * hs.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return RD_OK;
}

// The iterations between two checks: every scalar they need (alpha, beta,
// the live flags) is computed and read on the device, so the segment is one fixed
// sequence of launches.  B = 8 alternates the two direction buffers; `a` leaves with
// them in the order the next segment starts from.
rd_status cg_segment(CgArgs &a, int storage, int B, hipStream_t st, int iters)
{
    for (int k = 0; k < iters; ++k) {
        if (B == 8) {
            // p <- r + beta p fused into the matvec (beta = 0 on the first pass, where
            // p = r already), written to the other p buffer
            LAUNCHCHK(cg_launch_matvec_fused(storage, a, st));
            std::swap(a.p, a.p2);
        } else {
            // the same order: p <- r + beta p first (so that between iterations p is
            // the last direction and r the newest residual, as with B = 8)
            LAUNCHCHK(cg_launch_pupdate(storage, B, a, st));
            LAUNCHCHK(cg_launch_matvec(storage, B, a, st));
        }
        LAUNCHCHK(cg_launch_segsum(a, CG_PAP, -1, 0, st));
        LAUNCHCHK(cg_launch_update(storage, B, a, st));
        LAUNCHCHK(cg_launch_segsum(a, CG_RRNEW, CG_RRREC, 1, st));
    }
    return RD_OK;
}

// Segments captured once as hipGraphs (one per order of the two direction buffers) and
// replayed; kernels only (no memset nodes).
struct SegmentGraphs {
    hipStream_t cap = nullptr;
    struct Entry {
        void *p;
        int iters;
        hipGraphExec_t exec;
    };
    std::vector<Entry> g;
    ~SegmentGraphs()
    {
        for (auto &e : g) hipGraphExecDestroy(e.exec);
        if (cap) hipStreamDestroy(cap);
    }
    rd_status run(CgArgs &a, int storage, int B, hipStream_t st, int iters)
    {
        Entry *hit = nullptr;
        for (auto &e : g)
            if (e.p == a.p && e.iters == iters) hit = &e;
        if (!hit) {
            if (!cap) HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            CgArgs c = a;
            HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            rd_status s = cg_segment(c, storage, B, cap, iters);
            hipGraph_t graph = nullptr;
            const hipError_t ce = hipStreamEndCapture(cap, &graph);
            if (s != RD_OK) {
                if (graph) hipGraphDestroy(graph);
                return s;
            }
            HIPCHK(ce);
            Entry e{a.p, iters, nullptr};
            const hipError_t ie = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            HIPCHK(ie);
            g.push_back(e);
            hit = &g.back();
        }
        HIPCHK(hipGraphLaunch(hit->exec, st));
        if (B == 8 && (iters & 1)) std::swap(a.p, a.p2);
        return RD_OK;
    }
};

// Runs CG on every geometry of `a` (Dirichlet values already in x) from a linear
// ramp, stopping each geometry at rel. residual <= tol, stagnation or max_iters.
// check_every: iterations between two checks; use_graph: replay each segment of
// check_every iterations as a captured graph.
rd_status run_cg(const CgArgs &args, int storage, int B, hipStream_t st, int axis, double tol,
                 int64_t max_iters, const std::vector<GeomMeta> &meta, std::vector<CgOut> &out,
                 bool want_tau = true, int check_every = CHECK_EVERY, bool use_graph = true)
{
    const int stall_checks = std::max(1, STALL_ITERS / check_every);
    CgArgs a = args;  // B = 8 swaps the two p buffers every iteration
    const int n = a.ngeom;
    out.assign(n, CgOut());
    LAUNCHCHK(rd_launch_fill_u32(a.scal, 0u, (int64_t)n * CG_NSCAL * 2, st));
    if (!a.x64) return rd_fail(RD_ERR_STATE, "CG needs the FP64 iterate");
    if (B != 8) a.prec = 0;
    LAUNCHCHK(cg_launch_res64(storage, B, a, 1, st));
    LAUNCHCHK(cg_launch_segsum(a, CG_RRNEW, CG_BB, 2, st));
    if (a.prec > 0) {  // z = M^-1 r; CG_RR becomes r.z
        LAUNCHCHK(cg_launch_prec(storage, a, st));
        LAUNCHCHK(cg_launch_segsum(a, CG_RRNEW, CG_RRREC, 2, st));
    }
    std::vector<double> hs;
    rd_status s = copy_scal(a, hs, st);
    if (s != RD_OK) return s;
    std::vector<double> best(n, 0.0);
    std::vector<int> since(n, 0);
    int live = 0;
    for (int g = 0; g < n; ++g) {
        double *v = &hs[(size_t)g * CG_NSCAL];
        if (a.prec <= 0) v[CG_RRREC] = v[CG_RR];
        const double bb = v[CG_BB], rr = v[CG_RRREC];
        out[g].rel = bb > 0 ? sqrt(rr / bb) : 0.0;
        best[g] = out[g].rel;
        v[CG_SIGMA] = 1.0;
        v[CG_SIGMA_PREV] = 1.0;
        if (!(bb > 0) || out[g].rel <= tol || max_iters <= 0) {
            v[CG_DONE] = 1.0;
            out[g].converged = out[g].rel <= tol;
        } else {
            ++live;
        }
    }
    if ((s = push_scal(a, hs, st)) != RD_OK) return s;
    SegmentGraphs graphs;
    while (live > 0) {
        if (use_graph) {
            if ((s = graphs.run(a, storage, B, st, check_every)) != RD_OK) return s;
        } else {
            if ((s = cg_segment(a, storage, B, st, check_every)) != RD_OK) return s;
        }
        bool any = false;  // a geometry replaces or rescales its residual (CG_REPL)
        // true residual b - A x in FP64 (the recursive one drifts in the storage type's
        // precision); once the recursive residual has drifted from it, it replaces it
        // (residual replacement, van der Vorst and Ye 2000), so the iteration is not held
        // at the storage type's floor.  B = 8 reads the unfolded iterate; B = 4 folds
        // first.  The fold puts the updates of the last 25 iterations into X, clears x.
        if (B != 8 && !a.x64_direct) LAUNCHCHK(ir_launch_fold(storage, B, a, a.nb * (int64_t)B * B * B, st));
        LAUNCHCHK(cg_launch_res64(storage, B, a, 0, st));
        LAUNCHCHK(cg_launch_segsum(a, CG_CHECK, -1, -1, st));
        if (B == 8 && !a.x64_direct) LAUNCHCHK(ir_launch_fold(storage, B, a, a.nb * (int64_t)B * B * B, st));
        if ((s = copy_scal(a, hs, st)) != RD_OK) return s;
        for (int g = 0; g < n; ++g) {
            double *v = &hs[(size_t)g * CG_NSCAL];
            v[CG_REPL] = 0.0;
            if (v[CG_DONE] != 0.0) continue;
            out[g].iters += check_every;
            const double rel = sqrt(std::max(0.0, v[CG_CHECK]) / v[CG_BB]);
            out[g].rel = rel;
            if (!isfinite(rel)) return rd_fail(RD_ERR_NONFINITE, "CG residual is not finite");
            if (rel < 0.9 * best[g]) {
                best[g] = rel;
                since[g] = 0;
            } else {
                ++since[g];
            }
            const bool conv = rel <= tol;
            if (conv || since[g] >= stall_checks || out[g].iters >= max_iters) {
                v[CG_DONE] = 1.0;
                out[g].converged = conv;
                --live;
            } else {
                // next scale: a power of 2 that brings the residual's RMS near 1
                const double n_act = std::max(1.0, m_active(meta[g]));
                const double rms = sqrt(std::max(v[CG_CHECK], 1e-300) / n_act);
                // (only FP16 needs it: FP32 and BF16 have FP32's exponent range)
                const double sig = storage == RD_FP16
                                       ? ldexp(1.0, std::max(-60, std::min(60, (int)lround(-log2(rms)))))
                                       : 1.0;
                // replace the recursive residual once it has drifted from the true one by
                // more than a quarter (van der Vorst and Ye replace only where the gap
                // grows: every replacement costs the recursion some of its conjugacy)
                const double rec = sqrt(std::max(v[CG_RRREC], 0.0)) / v[CG_SIGMA];
                const double tru = sqrt(std::max(v[CG_CHECK], 0.0));
                const bool replace = fabs(rec - tru) > 0.25 * tru, rescale = sig != v[CG_SIGMA];
                v[CG_REPL] = replace ? 2.0 : rescale ? 3.0 : 0.0;  // this geometry's own choice
                // 16-bit vectors lose the directions' conjugacy over long runs (BF16 stalled
                // near 7.5e-7 on the 1024^3 foam without this): a replacement restarts the
                // direction (beta = 0: p = z next)
                if (replace && storage != RD_FP32) v[CG_BETA] = 0.0;
                any = any || replace || rescale;
                v[CG_SIGMA_PREV] = v[CG_SIGMA];  // what r and p hold until the kernel below
                v[CG_SIGMA] = sig;
            }
        }
        if ((s = push_scal(a, hs, st)) != RD_OK) return s;
        if (live > 0 && any) {
            // per geometry (CG_REPL): residual replacement, r = sigma (b - A X) in FP64 and
            // p rescaled, or only the rescaling of r and p; then rr of the stored r; the
            // other geometries of a batch keep their vectors and scalars
            LAUNCHCHK(cg_launch_res64(storage, B, a, 2, st));
            LAUNCHCHK(cg_launch_segsum(a, CG_RR, -1, -2, st));
            if (a.prec > 0) {  // and z = M^-1 r of the new r; CG_RR = r.z
                LAUNCHCHK(cg_launch_prec(storage, a, st));
                LAUNCHCHK(cg_launch_segsum(a, CG_RR, CG_RRREC, -2, st));
            }
        }
    }
    if (!want_tau) return RD_OK;
    // steady flux through the two Dirichlet planes (of the FP64 iterate rounded to x)
    LAUNCHCHK(ir_launch_store(storage, a.nb * (int64_t)B * B * B, a.x64, a.x, st));
    LAUNCHCHK(cg_launch_flux(B, a, 2 * axis, st));
    LAUNCHCHK(cg_launch_segsum(a, CG_QIN, CG_QOUT, -1, st));
    if ((s = copy_scal(a, hs, st)) != RD_OK) return s;
    for (int g = 0; g < n; ++g) {
        const GeomMeta &m = meta[g];
        const double *v = &hs[(size_t)g * CG_NSCAL];
        // the kernel sums (x_q - x_p) over Dirichlet-free pairs; the flux is D*dx times it
        out[g].qin = v[CG_QIN] * m.dx;
        out[g].qout = -v[CG_QOUT] * m.dx;
        const int64_t ext[3] = {m.nx, m.ny, m.nz};
        const double area = (double)ext[(axis + 1) % 3] * (double)ext[(axis + 2) % 3] * m.dx * m.dx;
        const double len = (double)(ext[axis] - 1) * m.dx;
        // inlet and outlet fluxes agree at an exact steady state; on an iterate their
        // mean is used (with BF16 / FP16 storage the inlet flux alone can vanish:
        // values just below 1 round to 1, while values near 0 keep their resolution)
        const double q = 0.5 * (out[g].qin + out[g].qout);
        out[g].tau = (m.percolates && q > 0) ? m.psi * area / (q * len)
                                              : std::numeric_limits<double>::infinity();
    }
    return RD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// single geometry
// ---------------------------------------------------------------------------

extern "C" rd_status rd_sim_steady_state(rd_sim *sim, int axis, double rel_tol, int64_t max_iters,
                                         double *tau, double *rel_residual, int64_t *iters)
{
    if (sim && sim->g->nparts() > 1)
        return rd_fail(RD_ERR_STATE, "rd_sim_steady_state: one geometry per simulation only");
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (!sim->ws) return rd_fail(RD_ERR_STATE, "bind a workspace first");
    if (!(sim->features & RD_WS_SOLVER))
        return rd_fail(RD_ERR_WORKSPACE, "bind with RD_WS_SOLVER for the steady state");
    if (sim->S != 1 || !sim->reactions.empty() || sim->robin[0] != 0.0)
        return rd_fail(RD_ERR_STATE, "steady state needs one species without reactions or Robin");
    if (sim->diff_path())
        return rd_fail(RD_ERR_STATE, "steady state needs a homogeneous D and no sink band (clear them)");
    if (axis < 0 || axis > 2) return rd_fail(RD_ERR_ARG, "axis must be 0, 1 or 2");
    if (!(rel_tol >= 0.0) || max_iters < 0) return rd_fail(RD_ERR_ARG, "bad tolerance or max_iters");
    const rd_geometry &G = *sim->g;
    const int64_t ext[3] = {G.nx, G.ny, G.nz};
    if (ext[axis] < 2) return rd_fail(RD_ERR_SHAPE, "need at least 2 voxels along the axis");
    const int inlet = 2 * axis, outlet = 2 * axis + 1;
    sim->dir[0] = (1u << inlet) | (1u << outlet);
    for (int f = 0; f < 6; ++f) sim->dirval[0][f] = 0.0;
    sim->dirval[0][inlet] = 1.0;
    sim->invalidate_graphs();
    CgArgs a{};
    a.info = (const BlockInfo *)(sim->ws + sim->L.info);
    a.mask = (const uint64_t *)(sim->ws + sim->L.mask);
    a.code = (const uint8_t *)(sim->ws + sim->L.code);
    a.geom = (const GeomInfo *)(sim->ws + sim->L.geom);
    a.nb = (int)G.nb();
    a.ngeom = 1;
    a.dir = sim->dir[0];
    a.x = sim->field_ptr(sim->cur, 0);
    a.r = sim->ws + sim->L.solver[0];
    a.p = sim->ws + sim->L.solver[1];
    a.ap = sim->ws + sim->L.solver[2];
    a.p2 = sim->ws + sim->L.solver[3];
    a.z = a.ap;  // free during CG with 8^3 blocks (A p is recomputed, never stored)
    a.prec = G.B == 8 ? sim->cg_prec : 0;
    a.partial = (double *)(sim->ws + sim->L.part);
    a.scal = (double *)(sim->ws + sim->L.scal);
    a.mid = (double *)(sim->ws + sim->L.mid);
    std::vector<GeomMeta> meta(1);
    meta[0] = {G.nx, G.ny, G.nz, (double)G.n_active / ((double)G.nx * G.ny * G.nz), G.dx, false};
    std::vector<CgOut> out;
    if (a.nb == 0) {
        if (tau) *tau = std::numeric_limits<double>::infinity();
        if (rel_residual) *rel_residual = 0.0;
        if (iters) *iters = 0;
        return RD_OK;
    }
    a.x64 = (double *)(sim->ws + sim->L.irx);  // the FP64 iterate (the guess writes it)
    {
        const size_t es = sim->storage == RD_FP32 ? 4 : 2;
        const SimLayout &L = sim->L;
        std::vector<char> perc;
        rd_status s = gpu_initial_guess(a, (int)sim->storage, G.B, axis, L.field_elems,
                                        L.solver[3] - L.solver[2] + es * (size_t)L.field_elems,
                                        L.solver[1] - L.solver[0], sim->stream, perc);
        if (s != RD_OK) return s;
        meta[0].percolates = perc[0] != 0;
    }
    // CG with an FP64 iterate X (starting at the guess) and FP64 residual replacement at
    // every check: direction and residual vectors stay in the storage type
    const int st_ = (int)sim->storage;
    const SimLayout &L = sim->L;
    const int64_t nslots = L.field_elems;
    hipStream_t stream = sim->stream;
    // FP32 storage: x accumulates the updates between checks (no FP64 traffic per
    // iteration); 16-bit storage is too coarse for that and updates X directly
    a.x64_direct = sim->storage == RD_FP32 ? 0 : 1;
    if (!a.x64_direct) LAUNCHCHK(rd_launch_fill_u32(a.x, 0u, nslots, stream));  // FP32: one word a slot
    rd_status s = run_cg(a, st_, G.B, stream, axis, rel_tol, max_iters, meta, out, true);
    if (s != RD_OK) return s;
    // (run_cg leaves X rounded to the storage type in the field and tau from its FP64 flux)
    const double rel = out[0].rel;
    const int64_t total = out[0].iters;
    const double t = out[0].tau;
    if (tau) *tau = t;
    if (rel_residual) *rel_residual = rel;
    if (iters) *iters = total;
    sim->steps_taken = 0;
    if (!out[0].converged)
        return rd_fail(RD_ERR_NOT_CONVERGED, "stopped at rel. residual " + std::to_string(rel));
    return RD_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------

struct rd_batch {
    std::vector<const rd_geometry *> geoms;
    rd_storage storage = RD_FP32;
    int B = 8;
    int64_t nb = 0;
    std::vector<BlockInfo> info;
    std::vector<uint64_t> mask;
    std::vector<uint8_t> code;
    std::vector<GeomInfo> ginfo;
    size_t o_info = 0, o_mask = 0, o_code = 0, o_geom = 0, o_vec[5] = {0, 0, 0, 0, 0}, o_x64 = 0, o_part = 0,
           o_scal = 0, total = 0;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    int check_every = CHECK_EVERY;  // CG iterations per captured segment / between checks
    bool use_graph = true;
    int cg_prec = 6;  // Jacobi steps of the block preconditioner (8^3 blocks; 0: plain CG)
};

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

extern "C" rd_status rd_batch_create(const rd_geometry *const *geoms, int n, rd_storage storage,
                                     rd_batch **out)
{
    if (!out) return rd_fail(RD_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!geoms || n <= 0 || n > 65535) return rd_fail(RD_ERR_ARG, "need 1..65535 geometries");
    if (storage != RD_FP32 && storage != RD_BF16 && storage != RD_FP16)
        return rd_fail(RD_ERR_ARG, "unknown storage type");
    const int B = geoms[0] ? geoms[0]->B : 0;
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        if (!geoms[i]) return rd_fail(RD_ERR_ARG, "NULL geometry");
        if (geoms[i]->B != B) return rd_fail(RD_ERR_SHAPE, "all geometries need the same block edge");
        total += geoms[i]->nb();
    }
    if (total >= INT32_MAX) return rd_fail(RD_ERR_SHAPE, "too many blocks in the batch");
    rd_batch *bt = new (std::nothrow) rd_batch();
    if (!bt) return rd_fail(RD_ERR_ARG, "out of host memory");
    bt->geoms.assign(geoms, geoms + n);
    bt->storage = storage;
    bt->B = B;
    bt->nb = total;
    const int MW = mask_words(B);
    try {
        bt->info.reserve(total);
        bt->mask.reserve((size_t)total * MW);
        bt->code.reserve((size_t)total * B * B * B);
        int32_t off = 0;
        int64_t dense = 0;
        for (int i = 0; i < n; ++i) {
            const rd_geometry &G = *geoms[i];
            if (G.nparts() > 1) throw std::invalid_argument("a batch member is a concatenation");
            bt->ginfo.push_back({(int32_t)G.nx, (int32_t)G.ny, (int32_t)G.nz, off, dense});
            dense += G.dense_size();
            for (int64_t b = 0; b < G.nb(); ++b) {
                BlockInfo bi = G.info[b];
                for (int f = 0; f < 6; ++f)
                    if (bi.nbr[f] >= 0) bi.nbr[f] += off;
                bi.zg = (bi.zg & 0xffff) | (i << 16);
                bt->info.push_back(bi);
            }
            bt->mask.insert(bt->mask.end(), G.mask.begin(), G.mask.end());
            bt->code.insert(bt->code.end(), G.code.begin(), G.code.end());
            off += (int32_t)G.nb();
        }
    } catch (const std::bad_alloc &) {
        delete bt;
        return rd_fail(RD_ERR_ARG, "out of host memory");
    } catch (const std::invalid_argument &e) {
        delete bt;
        return rd_fail(RD_ERR_ARG, e.what());
    }
    const size_t es = storage == RD_FP32 ? 4 : 2;
    const size_t nbs = (size_t)std::max<int64_t>(total, 1);
    size_t o = 0;
    bt->o_info = o; o = al256(o + sizeof(BlockInfo) * nbs);
    bt->o_mask = o; o = al256(o + 8 * (size_t)MW * nbs);
    bt->o_code = o; o = al256(o + nbs * (size_t)B * B * B);
    bt->o_geom = o; o = al256(o + sizeof(GeomInfo) * (size_t)n);
    for (int v = 0; v < 5; ++v) {  // x, r, p, Ap, second p
        bt->o_vec[v] = o;
        o = al256(o + es * nbs * (size_t)B * B * B);
    }
    bt->o_x64 = o; o = al256(o + sizeof(double) * nbs * (size_t)B * B * B);  // FP64 iterate
    bt->o_part = o; o = al256(o + sizeof(double) * 2 * nbs);
    bt->o_scal = o; o = al256(o + sizeof(double) * CG_NSCAL * (size_t)n);
    bt->total = o;
    *out = bt;
    return RD_OK;
}

extern "C" rd_status rd_batch_workspace_bytes(const rd_batch *b, size_t *bytes)
{
    if (!b || !bytes) return rd_fail(RD_ERR_ARG, "NULL argument");
    *bytes = b->total;
    return RD_OK;
}

extern "C" rd_status rd_batch_bind(rd_batch *b, void *dev_ws, size_t bytes, void *stream)
{
    if (!b) return rd_fail(RD_ERR_ARG, "batch is NULL");
    if (!dev_ws) return rd_fail(RD_ERR_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)dev_ws) % 256) return rd_fail(RD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    if (bytes < b->total)
        return rd_fail(RD_ERR_WORKSPACE, "workspace has " + std::to_string(bytes) + " bytes, needs " +
                                             std::to_string(b->total));
    b->ws = (char *)dev_ws;
    b->stream = (hipStream_t)stream;
    if (b->nb > 0) {
        HIPCHK(hipMemcpyAsync(b->ws + b->o_info, b->info.data(), sizeof(BlockInfo) * b->nb,
                              hipMemcpyHostToDevice, b->stream));
        HIPCHK(hipMemcpyAsync(b->ws + b->o_mask, b->mask.data(), sizeof(uint64_t) * b->mask.size(),
                              hipMemcpyHostToDevice, b->stream));
        HIPCHK(hipMemcpyAsync(b->ws + b->o_code, b->code.data(), b->code.size(), hipMemcpyHostToDevice,
                              b->stream));
    }
    HIPCHK(hipMemcpyAsync(b->ws + b->o_geom, b->ginfo.data(), sizeof(GeomInfo) * b->ginfo.size(),
                          hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return RD_OK;
}

namespace {
// Labelling, initial guess and CG of every geometry of a bound batch (want_tau: the flux
// and tau at the end).
rd_status batch_cg(rd_batch *b, int axis, double rel_tol, int64_t max_iters, bool want_tau,
                   std::vector<CgOut> &out)
{
    if (!b) return rd_fail(RD_ERR_ARG, "batch is NULL");
    if (!b->ws) return rd_fail(RD_ERR_STATE, "bind a workspace first");
    if (axis < 0 || axis > 2) return rd_fail(RD_ERR_ARG, "axis must be 0, 1 or 2");
    const int n = (int)b->geoms.size();
    std::vector<GeomMeta> meta(n);
    for (int i = 0; i < n; ++i) {
        const rd_geometry &G = *b->geoms[i];
        const int64_t ext[3] = {G.nx, G.ny, G.nz};
        if (ext[axis] < 2) return rd_fail(RD_ERR_SHAPE, "need at least 2 voxels along the axis");
        meta[i] = {G.nx, G.ny, G.nz, (double)G.n_active / ((double)G.nx * G.ny * G.nz), G.dx, false};
    }
    const int inlet = 2 * axis, outlet = 2 * axis + 1;
    const size_t es = b->storage == RD_FP32 ? 4 : 2;
    const size_t NS = (size_t)b->B * b->B * b->B;
    CgArgs a{};
    a.info = (const BlockInfo *)(b->ws + b->o_info);
    a.mask = (const uint64_t *)(b->ws + b->o_mask);
    a.code = (const uint8_t *)(b->ws + b->o_code);
    a.geom = (const GeomInfo *)(b->ws + b->o_geom);
    a.nb = (int)b->nb;
    a.ngeom = n;
    a.dir = (1u << inlet) | (1u << outlet);
    a.x = b->ws + b->o_vec[0];
    a.r = b->ws + b->o_vec[1];
    a.p = b->ws + b->o_vec[2];
    a.ap = b->ws + b->o_vec[3];
    a.p2 = b->ws + b->o_vec[4];
    a.z = a.ap;
    a.prec = b->B == 8 ? b->cg_prec : 0;
    a.partial = (double *)(b->ws + b->o_part);
    a.scal = (double *)(b->ws + b->o_scal);
    if (b->nb > 0) {
        std::vector<char> perc;
        const int64_t nslots = b->nb * (int64_t)NS;
        a.x64 = (double *)(b->ws + b->o_x64);  // the FP64 iterate (the guess writes it)
        rd_status s0 = gpu_initial_guess(a, (int)b->storage, b->B, axis, nslots,
                                         b->o_vec[4] - b->o_vec[3] + es * (size_t)nslots,
                                         b->o_vec[2] - b->o_vec[1], b->stream, perc);
        if (s0 != RD_OK) return s0;
        for (int i = 0; i < n; ++i) meta[i].percolates = perc[(size_t)i] != 0;
        // FP64 iterate with residual replacement, as for one geometry
        a.x64_direct = b->storage == RD_FP32 ? 0 : 1;
        if (!a.x64_direct) LAUNCHCHK(rd_launch_fill_u32(a.x, 0u, nslots, b->stream));
        return run_cg(a, (int)b->storage, b->B, b->stream, axis, rel_tol, max_iters, meta, out,
                      want_tau, b->check_every, b->use_graph);
    }
    out.assign(n, CgOut());
    for (auto &o : out) o.tau = std::numeric_limits<double>::infinity();
    return RD_OK;
}
}  // namespace

extern "C" rd_status rd_batch_tortuosity(rd_batch *b, int axis, double rel_tol, int64_t max_iters,
                                         double *tau, double *rel_residual, int64_t *iters)
{
    std::vector<CgOut> out;
    rd_status s = batch_cg(b, axis, rel_tol, max_iters, true, out);
    if (s != RD_OK) return s;
    const int n = (int)b->geoms.size();
    bool all = true;
    for (int i = 0; i < n; ++i) {
        if (tau) tau[i] = out[i].tau;
        if (rel_residual) rel_residual[i] = out[i].rel;
        if (iters) iters[i] = out[i].iters;
        all = all && out[i].converged;
    }
    if (!all) return rd_fail(RD_ERR_NOT_CONVERGED, "some geometries stopped above the tolerance");
    return RD_OK;
}

extern "C" rd_status rd_batch_set_launch(rd_batch *b, int iters_per_check, int use_graph)
{
    if (!b) return rd_fail(RD_ERR_ARG, "batch is NULL");
    if (iters_per_check < 1 || iters_per_check > 1000) return rd_fail(RD_ERR_ARG, "iters_per_check in 1..1000");
    b->check_every = iters_per_check;
    b->use_graph = use_graph != 0;
    return RD_OK;
}

extern "C" rd_status rd_sim_set_cg_precond(rd_sim *sim, int jacobi_steps)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (jacobi_steps < 0 || jacobi_steps > 16) return rd_fail(RD_ERR_ARG, "jacobi_steps must be 0..16");
    sim->cg_prec = jacobi_steps;
    return RD_OK;
}

extern "C" rd_status rd_batch_set_cg_precond(rd_batch *b, int jacobi_steps)
{
    if (!b) return rd_fail(RD_ERR_ARG, "batch is NULL");
    if (jacobi_steps < 0 || jacobi_steps > 16) return rd_fail(RD_ERR_ARG, "jacobi_steps must be 0..16");
    b->cg_prec = jacobi_steps;
    return RD_OK;
}

extern "C" rd_status rd_batch_get_launch(const rd_batch *b, int *iters_per_check, int *use_graph)
{
    if (!b) return rd_fail(RD_ERR_ARG, "batch is NULL");
    if (iters_per_check) *iters_per_check = b->check_every;
    if (use_graph) *use_graph = b->use_graph ? 1 : 0;
    return RD_OK;
}

namespace {
// Wall time per iteration of trial_iters CG iterations of a batch with its current launch
// setting: a run with them minus one without (labelling, initial guess and the first
// residual are in both; a first run without iterations warms the launch paths up).
rd_status batch_ms_per_iter(rd_batch *b, int axis, int64_t trial_iters, double *ms)
{
    std::vector<CgOut> out;
    rd_status s = batch_cg(b, axis, 0.0, 0, false, out);
    if (s != RD_OK) return s;
    auto t0 = std::chrono::steady_clock::now();
    s = batch_cg(b, axis, 0.0, 0, false, out);
    if (s != RD_OK) return s;
    auto t1 = std::chrono::steady_clock::now();
    s = batch_cg(b, axis, 0.0, trial_iters, false, out);
    if (s != RD_OK) return s;
    auto t2 = std::chrono::steady_clock::now();
    int64_t done = 0;
    for (const CgOut &o : out) done = std::max(done, o.iters);
    *ms = std::max(1e-6, std::chrono::duration<double, std::milli>((t2 - t1) - (t1 - t0)).count() /
                             (double)std::max<int64_t>(1, done));
    return RD_OK;
}
}  // namespace

extern "C" rd_status rd_batch_autotune_pick(rd_batch *const *batches, int n, int axis, int64_t trial_iters,
                                            int *best_index, double *ms_per_iter)
{
    if (!batches || n <= 0 || !best_index) return rd_fail(RD_ERR_ARG, "need batches and best_index");
    if (trial_iters < 1) return rd_fail(RD_ERR_ARG, "trial_iters >= 1");
    *best_index = -1;
    double best = 1e300;
    for (int i = 0; i < n; ++i) {
        // each candidate keeps its fastest launch setting: iterations per captured
        // segment (between residual checks) and graph replay or direct launches
        rd_batch *b = batches[i];
        if (!b) return rd_fail(RD_ERR_ARG, "NULL batch");
        double bi = 1e300;
        int bc = b->check_every;
        bool bg = b->use_graph;
        for (int ce : {25, 50})
            for (int gr = 1; gr >= 0; --gr) {
                b->check_every = ce;
                b->use_graph = gr != 0;
                double ms = 0.0;
                rd_status s = batch_ms_per_iter(b, axis, std::max<int64_t>(trial_iters, ce), &ms);
                if (s != RD_OK) return s;
                if (ms < bi) {
                    bi = ms;
                    bc = ce;
                    bg = gr != 0;
                }
            }
        b->check_every = bc;
        b->use_graph = bg;
        if (ms_per_iter) ms_per_iter[i] = bi;
        if (bi < best) {
            best = bi;
            *best_index = i;
        }
    }
    return RD_OK;
}

extern "C" void rd_batch_destroy(rd_batch *b) { delete b; }

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------

// Checkpointed adjoint: a forward sweep stores c^{jk} every k steps; the backward
// sweep restores each segment's first state, recomputes the segment's states into
// k-1 spare slots with the same step kernel (bitwise the forward states) and runs
// the adjoint steps from the segment's end to its start.
static rd_status adjoint_impl(rd_sim *sim, const float *dev_seed, int seed_mode, int64_t n_steps, double dt,
                              int checkpoint_every, double *loss, double *dL_dD, double *dL_drate,
                              double *dev_dL_de)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (!sim->ws) return rd_fail(RD_ERR_STATE, "bind a workspace first");
    if (!(sim->features & RD_WS_ADJOINT))
        return rd_fail(RD_ERR_WORKSPACE, "bind with RD_WS_ADJOINT for the adjoint");
    if (sim->S != 1) return rd_fail(RD_ERR_STATE, "the adjoint needs a single species");
    if (sim->sink_active()) return rd_fail(RD_ERR_STATE, "the adjoint does not cover the sink band (clear it)");
    const bool fac = sim->diff_on;
    if (dev_dL_de && !fac) return rd_fail(RD_ERR_STATE, "dL/de needs a diffusivity factor (rd_sim_set_diffusivity)");
    for (const Reaction &r : sim->reactions)
        if (r.to != -1) return rd_fail(RD_ERR_STATE, "the adjoint supports decay reactions only");
    if (sim->sround)
        return rd_fail(RD_ERR_STATE, "the adjoint needs round-to-nearest storage");
    if (!dev_seed) return rd_fail(RD_ERR_ARG, "seed field is NULL");
    if (seed_mode != 0 && seed_mode != 1) return rd_fail(RD_ERR_ARG, "seed_mode must be 0 or 1");
    if (n_steps < 1 || checkpoint_every < 1) return rd_fail(RD_ERR_ARG, "need n_steps, checkpoint_every >= 1");
    rd_status s = sim->check_dt(dt);
    if (s != RD_OK) return s;
    const int64_t k = checkpoint_every;
    const int64_t ncp = (n_steps + k - 1) / k;
    if (ncp + k - 1 > sim->cp_slots)
        return rd_fail(RD_ERR_WORKSPACE, "need " + std::to_string(ncp + k - 1) +
                                             " checkpoint slots, the workspace has " +
                                             std::to_string(sim->cp_slots));
    const rd_geometry &G = *sim->g;
    const int B = G.B, nb = (int)G.nb();
    const int st = (int)sim->storage;
    hipStream_t stream = sim->stream;
    const size_t es = sim->storage == RD_FP32 ? 4 : 2;
    const size_t fbytes = es * (size_t)sim->L.field_elems;
    char *ws = sim->ws;
    auto slot = [&](int64_t j) { return (void *)(ws + sim->L.cp + sim->L.cp_stride * (size_t)j); };
    double *acc = (double *)(ws + sim->L.res) + 16;  // [loss, gD, gk]
    LAUNCHCHK(rd_launch_fill_u32(acc, 0u, 6, stream));
    const int64_t ndense = G.nx * G.ny * G.nz;
    if (nb == 0) {
        if (loss) *loss = 0;
        if (dL_dD) *dL_dD = 0;
        if (dL_drate) *dL_drate = 0;
        if (dev_dL_de) LAUNCHCHK(rd_launch_fill_u32(dev_dL_de, 0u, 2 * ndense, stream));
        return RD_OK;
    }
    double *ge = fac ? (double *)(ws + sim->L.ge) : nullptr;
    if (fac) LAUNCHCHK(rd_launch_fill_u32(ge, 0u, 2 * sim->L.field_elems, stream));
    const float *efac = (const float *)(ws + sim->L.diff);
    // the seed in block-major FP32
    float zero6[6] = {0, 0, 0, 0, 0, 0};
    float *seed = (float *)(ws + sim->L.target);
    LAUNCHCHK(rd_launch_scatter(0, B, (const BlockInfo *)(ws + sim->L.info),
                                (const uint64_t *)(ws + sim->L.mask), nullptr, (const GeomInfo *)(ws + sim->L.geom),
                                nb, dev_seed, seed, 0u, zero6, stream));
    // forward with checkpoints
    for (int64_t j = 0; j < ncp; ++j) {
        HIPCHK(hipMemcpyAsync(slot(j), sim->field_ptr(sim->cur, 0), fbytes, hipMemcpyDeviceToDevice, stream));
        s = sim->step(dt, std::min<int64_t>(k, n_steps - j * k));
        if (s != RD_OK) return s;
    }
    AdjArgs a{};
    a.info = (const BlockInfo *)(ws + sim->L.info);
    a.mask = (const uint64_t *)(ws + sim->L.mask);
    a.code = (const uint8_t *)(ws + sim->L.code);
    a.geom = (const GeomInfo *)(ws + sim->L.geom);
    a.nb = nb;
    const StepArgs fa = sim->step_args(dt, sim->cur);
    a.coef = fa.coef[0];
    a.seed = seed;
    a.partial = (double *)(ws + sim->L.part);
    float *lam[2] = {(float *)(ws + sim->L.lam[0]), (float *)(ws + sim->L.lam[1])};
    int lc = 0;
    // lambda^N
    a.c = sim->field_ptr(sim->cur, 0);
    a.lam_out = lam[lc];
    LAUNCHCHK(adj_launch_seed(st, B, a, seed_mode, stream));
    double *mid = (double *)(ws + sim->L.mid);
    LAUNCHCHK(rd_launch_finish_reduce(a.partial, nb, 1, mid, acc, stream));
    // the step kernel adds its gradient terms to its own FP64 rows, in step order; one
    // fixed-order reduction over the rows after the sweep
    const int nrows = adj_groups(B, nb);
    LAUNCHCHK(rd_launch_fill_u32(a.partial, 0u, (int64_t)nrows * 4, stream));
    // backward over segments
    for (int64_t j = ncp - 1; j >= 0; --j) {
        const int64_t s0 = j * k;
        const int64_t len = std::min<int64_t>(k, n_steps - s0);
        // seg[0] = checkpoint j, seg[m] = spare slot ncp + m - 1
        auto seg = [&](int64_t m) { return m == 0 ? slot(j) : slot(ncp + m - 1); };
        for (int64_t m = 1; m < len; ++m) {
            StepArgs sa = fa;
            sa.cin = seg(m - 1);
            sa.cout = seg(m);
            sa.sround = 0;
            sa.ctr = sim->step_counter();
            sa.ctr_off = 0;
            sim->launch_shape(sa);
            if (fac) {  // the inhomogeneous step, as rd_sim_step runs it
                const int column = B == 8 && sim->kernel != 0 ? 1 : 0;
                sa.xcd_chunk = 0;
                DiffArgs da{sa, efac, {0.0f, 0.0f, 0.0f, 0.0f}};
                LAUNCHCHK(rd_launch_step_diff(st, B, da, column, stream));
            } else {
                LAUNCHCHK(rd_launch_step(st, B, sa, stream));
            }
        }
        for (int64_t m = len - 1; m >= 0; --m) {
            a.c = seg(m);
            a.lam_in = lam[lc];
            a.lam_out = lam[1 - lc];
            if (fac) {
                AdjEArgs x{a, efac, sim->D[0] * dt / (G.dx * G.dx), ge};
                LAUNCHCHK(adj_launch_step_e(st, B, x, B == 8 && sim->kernel != 0 ? 1 : 0, stream));
            } else {
                LAUNCHCHK(adj_launch_step(st, B, a, stream));
            }
            lc = 1 - lc;
        }
    }
    LAUNCHCHK(rd_launch_finish_reduce(a.partial, nrows, 2, mid, acc + 1, stream));
    if (dev_dL_de)
        LAUNCHCHK(adj_launch_dense_f64(B, a.info, a.code, a.geom, nb, ge, dev_dL_de, ndense, stream));
    double h[3];
    HIPCHK(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    const double dx = G.dx;
    if (loss) *loss = seed_mode == 0 ? h[0] : 0.0;
    if (dL_dD) *dL_dD = h[1] * dt / (dx * dx);
    if (dL_drate) *dL_drate = h[2] * dt;
    if (!isfinite(h[0]) || !isfinite(h[1]) || !isfinite(h[2]))
        return rd_fail(RD_ERR_NONFINITE, "adjoint produced a non-finite value");
    return RD_OK;
}

extern "C" rd_status rd_sim_adjoint(rd_sim *sim, const float *dev_seed, int seed_mode, int64_t n_steps, double dt,
                                    int checkpoint_every, double *loss, double *dL_dD, double *dL_drate)
{
    if (sim && sim->g->nparts() > 1)
        return rd_fail(RD_ERR_STATE, "rd_sim_adjoint: one geometry per simulation only");
    return adjoint_impl(sim, dev_seed, seed_mode, n_steps, dt, checkpoint_every, loss, dL_dD, dL_drate, nullptr);
}

extern "C" rd_status rd_sim_adjoint_factor(rd_sim *sim, const float *dev_seed, int seed_mode, int64_t n_steps,
                                           double dt, int checkpoint_every, double *loss, double *dL_dD,
                                           double *dL_drate, double *dev_dL_de)
{
    if (sim && sim->g->nparts() > 1)
        return rd_fail(RD_ERR_STATE, "rd_sim_adjoint_factor: one geometry per simulation only");
    if (!dev_dL_de) return rd_fail(RD_ERR_ARG, "dL/de output is NULL");
    if (sim && !(sim->features & RD_WS_DIFFUSIVITY))
        return rd_fail(RD_ERR_WORKSPACE, "bind with RD_WS_ADJOINT | RD_WS_DIFFUSIVITY for dL/de");
    return adjoint_impl(sim, dev_seed, seed_mode, n_steps, dt, checkpoint_every, loss, dL_dD, dL_drate, dev_dL_de);
}

extern "C" rd_status rd_sim_set_species_D(rd_sim *sim, int species, double D)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (species < 0 || species >= sim->S) return rd_fail(RD_ERR_ARG, "bad species");
    if (!(D >= 0.0) || !isfinite(D)) return rd_fail(RD_ERR_ARG, "D must be finite and >= 0");
    sim->D[species] = D;
    sim->invalidate_graphs();
    return RD_OK;
}

extern "C" rd_status rd_sim_set_reaction_rate(rd_sim *sim, int index, double rate)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (index < 0 || index >= (int)sim->reactions.size()) return rd_fail(RD_ERR_ARG, "bad reaction index");
    if (!(rate >= 0.0) || !isfinite(rate)) return rd_fail(RD_ERR_ARG, "rate must be finite and >= 0");
    sim->reactions[index].rate = rate;
    sim->invalidate_graphs();
    return RD_OK;
}
