// rd_api.cpp -- the C ABI: validation, workspace layout, launch driver, reductions.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>

#include "rd_host.h"
#include "rd_diff.h"
#include "rd_sim.h"

static thread_local std::string g_last_error;

rd_status rd_fail(rd_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

extern "C" const char *rd_status_string(rd_status s)
{
    switch (s) {
    case RD_OK: return "ok";
    case RD_ERR_ARG: return "bad argument";
    case RD_ERR_SHAPE: return "bad shape";
    case RD_ERR_INCONSISTENT_SDF: return "sdf sign disagrees with image";
    case RD_ERR_UNSTABLE_DT: return "time step above the stability bound";
    case RD_ERR_WORKSPACE: return "workspace missing or too small";
    case RD_ERR_HIP: return "HIP runtime error";
    case RD_ERR_NONFINITE: return "non-finite value in field";
    case RD_ERR_NOT_CONVERGED: return "not converged";
    case RD_ERR_STATE: return "call out of order";
    }
    return "unknown status";
}

extern "C" const char *rd_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------

extern "C" rd_status rd_geometry_create(const uint8_t *image, const float *sdf, int64_t nx,
                                        int64_t ny, int64_t nz, double dx, int block_edge,
                                        rd_geometry **out)
{
    if (!out) return rd_fail(RD_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!image) return rd_fail(RD_ERR_ARG, "image is NULL");
    if (nx <= 0 || ny <= 0 || nz <= 0) return rd_fail(RD_ERR_SHAPE, "non-positive extent");
    if (nx > 65535L * 8 || ny > 65535L * 8 || nz > 65535L * 8 || nx * ny > ((int64_t)1 << 40))
        return rd_fail(RD_ERR_SHAPE, "volume too large");
    if (nx >= INT32_MAX || ny >= INT32_MAX || nz >= INT32_MAX)
        return rd_fail(RD_ERR_SHAPE, "extent does not fit int32");
    if (block_edge != 4 && block_edge != 8) return rd_fail(RD_ERR_SHAPE, "block_edge must be 4 or 8");
    if (!(dx > 0.0) || !isfinite(dx)) return rd_fail(RD_ERR_ARG, "dx must be positive");
    const int64_t N = nx * ny * nz;
    if (sdf) {
        for (int64_t i = 0; i < N; ++i) {
            const bool in = image[i] != 0;
            if ((sdf[i] > 0.0f) != in) {
                const int64_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
                return rd_fail(RD_ERR_INCONSISTENT_SDF,
                               "sdf > 0 disagrees with image at (x,y,z) = (" + std::to_string(x) +
                                   "," + std::to_string(y) + "," + std::to_string(z) + ")");
            }
        }
    }
    rd_geometry *g = new (std::nothrow) rd_geometry();
    if (!g) return rd_fail(RD_ERR_ARG, "out of host memory");
    g->dx = dx;
    rd_status s;
    try {
        s = rd_geometry_build(image, nx, ny, nz, block_edge, g);
    } catch (const std::bad_alloc &) {
        s = rd_fail(RD_ERR_ARG, "out of host memory");
    }
    if (s != RD_OK) {
        delete g;
        return s;
    }
    *out = g;
    return RD_OK;
}

extern "C" rd_status rd_geometry_stats(const rd_geometry *g, int64_t *n_active_vox,
                                       int64_t *n_active_blocks, double *porosity, double *fill)
{
    if (!g) return rd_fail(RD_ERR_ARG, "geometry is NULL");
    const int64_t nb = g->nb();
    const double slots = (double)nb * g->B * g->B * g->B;
    if (n_active_vox) *n_active_vox = g->n_active;
    if (n_active_blocks) *n_active_blocks = nb;
    if (porosity) *porosity = (double)g->n_active / ((double)g->nx * g->ny * g->nz);
    if (fill) *fill = nb ? (double)g->n_active / slots : 0.0;
    return RD_OK;
}

extern "C" rd_status rd_geometry_export_index(const rd_geometry *g, int64_t *block_id, int32_t *nbr)
{
    if (!g) return rd_fail(RD_ERR_ARG, "geometry is NULL");
    const int64_t nb = g->nb();
    if (block_id) memcpy(block_id, g->block_id.data(), sizeof(int64_t) * nb);
    if (nbr)
        for (int64_t b = 0; b < nb; ++b)
            for (int f = 0; f < 6; ++f) nbr[b * 6 + f] = g->info[b].nbr[f];
    return RD_OK;
}

extern "C" rd_status rd_geometry_export_masks(const rd_geometry *g, uint64_t *masks)
{
    if (!g || !masks) return rd_fail(RD_ERR_ARG, "NULL argument");
    const int own = g->B == 8 ? 8 : 1, MW = mask_words(g->B);
    for (int64_t b = 0; b < g->nb(); ++b)
        for (int w = 0; w < own; ++w) masks[b * own + w] = g->mask[b * MW + w];
    return RD_OK;
}

extern "C" rd_status rd_geometry_export_codes(const rd_geometry *g, uint8_t *codes)
{
    if (!g || !codes) return rd_fail(RD_ERR_ARG, "NULL argument");
    memcpy(codes, g->code.data(), g->code.size());
    return RD_OK;
}

extern "C" rd_status rd_geometry_concat(const rd_geometry *const *geoms, int n, rd_geometry **out)
{
    if (!out) return rd_fail(RD_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!geoms || n <= 0 || n > 65535) return rd_fail(RD_ERR_ARG, "need 1..65535 geometries");
    for (int i = 0; i < n; ++i) {
        if (!geoms[i]) return rd_fail(RD_ERR_ARG, "NULL geometry");
        if (geoms[i]->nparts() > 1) return rd_fail(RD_ERR_ARG, "a part is itself a concatenation");
        if (geoms[i]->B != geoms[0]->B) return rd_fail(RD_ERR_SHAPE, "all parts need the same block edge");
        if (geoms[i]->dx != geoms[0]->dx) return rd_fail(RD_ERR_SHAPE, "all parts need the same dx");
    }
    int64_t total = 0, dense = 0;
    for (int i = 0; i < n; ++i) total += geoms[i]->nb();
    if (total >= INT32_MAX) return rd_fail(RD_ERR_SHAPE, "too many blocks");
    rd_geometry *g = new (std::nothrow) rd_geometry();
    if (!g) return rd_fail(RD_ERR_ARG, "out of host memory");
    const int B = geoms[0]->B, MW = mask_words(B);
    g->B = B;
    g->dx = geoms[0]->dx;
    try {
        g->block_id.reserve(total);
        g->info.reserve(total);
        g->mask.reserve((size_t)total * MW);
        g->code.reserve((size_t)total * B * B * B);
        int32_t off = 0;
        for (int i = 0; i < n; ++i) {
            const rd_geometry &G = *geoms[i];
            g->parts.push_back({(int32_t)G.nx, (int32_t)G.ny, (int32_t)G.nz, off, dense});
            for (int64_t b = 0; b < G.nb(); ++b) {
                BlockInfo bi = G.info[b];
                for (int f = 0; f < 6; ++f)
                    if (bi.nbr[f] >= 0) bi.nbr[f] += off;
                bi.zg = (bi.zg & 0xffff) | (i << 16);
                g->info.push_back(bi);
            }
            g->block_id.insert(g->block_id.end(), G.block_id.begin(), G.block_id.end());
            g->mask.insert(g->mask.end(), G.mask.begin(), G.mask.end());
            g->code.insert(g->code.end(), G.code.begin(), G.code.end());
            g->n_active += G.n_active;
            off += (int32_t)G.nb();
            dense += G.dense_size();
        }
    } catch (const std::bad_alloc &) {
        delete g;
        return rd_fail(RD_ERR_ARG, "out of host memory");
    }
    g->nx = dense;
    g->ny = g->nz = 1;
    *out = g;
    return RD_OK;
}

extern "C" rd_status rd_geometry_part_info(const rd_geometry *g, int part, int64_t shape[3], int64_t *dense_offset,
                                           int64_t *first_block, int64_t *n_blocks)
{
    if (!g) return rd_fail(RD_ERR_ARG, "geometry is NULL");
    if (part < 0 || part >= g->nparts()) return rd_fail(RD_ERR_ARG, "bad part");
    if (g->parts.empty()) {
        if (shape) shape[0] = g->nz, shape[1] = g->ny, shape[2] = g->nx;
        if (dense_offset) *dense_offset = 0;
        if (first_block) *first_block = 0;
        if (n_blocks) *n_blocks = g->nb();
        return RD_OK;
    }
    const GeomInfo &p = g->parts[part];
    const int64_t end = part + 1 < g->nparts() ? g->parts[part + 1].block0 : g->nb();
    if (shape) shape[0] = p.nz, shape[1] = p.ny, shape[2] = p.nx;
    if (dense_offset) *dense_offset = p.dense0;
    if (first_block) *first_block = p.block0;
    if (n_blocks) *n_blocks = end - p.block0;
    return RD_OK;
}

extern "C" int rd_geometry_parts(const rd_geometry *g) { return g ? g->nparts() : 0; }

extern "C" void rd_geometry_destroy(rd_geometry *g) { delete g; }

// ---------------------------------------------------------------------------
// simulation set-up
// ---------------------------------------------------------------------------

extern "C" rd_status rd_sim_create(const rd_geometry *g, rd_storage storage, rd_sim **out)
{
    if (!out) return rd_fail(RD_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!g) return rd_fail(RD_ERR_ARG, "geometry is NULL");
    if (storage != RD_FP32 && storage != RD_BF16 && storage != RD_FP16)
        return rd_fail(RD_ERR_ARG, "unknown storage type");
    rd_sim *s = new (std::nothrow) rd_sim();
    if (!s) return rd_fail(RD_ERR_ARG, "out of host memory");
    s->g = g;
    s->storage = storage;
    *out = s;
    return RD_OK;
}

extern "C" rd_status rd_sim_add_species(rd_sim *sim, double D, int *id)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (sim->ws) return rd_fail(RD_ERR_STATE, "species must be added before rd_sim_bind");
    if (sim->S >= RD_MAX_SPECIES) return rd_fail(RD_ERR_ARG, "at most 4 species");
    if (!(D >= 0.0) || !isfinite(D)) return rd_fail(RD_ERR_ARG, "D must be finite and >= 0");
    sim->D[sim->S] = D;
    if (id) *id = sim->S;
    sim->S++;
    return RD_OK;
}

extern "C" rd_status rd_sim_add_reaction(rd_sim *sim, int from, int to, double rate)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (from < 0 || from >= sim->S) return rd_fail(RD_ERR_ARG, "bad 'from' species");
    if (to < -1 || to >= sim->S || to == from) return rd_fail(RD_ERR_ARG, "bad 'to' species");
    if (!(rate >= 0.0) || !isfinite(rate)) return rd_fail(RD_ERR_ARG, "rate must be finite and >= 0");
    sim->reactions.push_back({from, to, rate});
    sim->invalidate_graphs();
    return RD_OK;
}

extern "C" rd_status rd_sim_set_robin(rd_sim *sim, int species, double k)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (species < 0 || species >= sim->S) return rd_fail(RD_ERR_ARG, "bad species");
    if (!(k >= 0.0) || !isfinite(k)) return rd_fail(RD_ERR_ARG, "k must be finite and >= 0");
    sim->robin[species] = k;
    sim->invalidate_graphs();
    return RD_OK;
}

extern "C" rd_status rd_sim_set_dirichlet(rd_sim *sim, int species, int face, double value)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (species < 0 || species >= sim->S) return rd_fail(RD_ERR_ARG, "bad species");
    if (face < 0 || face > 5) return rd_fail(RD_ERR_ARG, "face must be 0..5");
    if (!isfinite(value)) return rd_fail(RD_ERR_ARG, "value must be finite");
    sim->dir[species] |= 1u << face;
    sim->dirval[species][face] = value;
    sim->invalidate_graphs();
    if (sim->ws) return sim->apply_dirichlet(species);
    return RD_OK;
}

extern "C" rd_status rd_sim_clear_dirichlet(rd_sim *sim, int species)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (species < 0 || species >= sim->S) return rd_fail(RD_ERR_ARG, "bad species");
    sim->dir[species] = 0;
    sim->invalidate_graphs();
    return RD_OK;
}

extern "C" rd_status rd_sim_set_launch(rd_sim *sim, int graph_steps, int use_graph, int xcd_map)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (graph_steps < 1 || graph_steps > 4096) return rd_fail(RD_ERR_ARG, "graph_steps in 1..4096");
    sim->graph_steps = graph_steps;
    sim->use_graph = use_graph != 0;
    sim->xcd_map = xcd_map != 0;
    sim->invalidate_graphs();
    return RD_OK;
}

extern "C" rd_status rd_sim_set_layout(rd_sim *sim, int layout)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (layout != RD_LAYOUT_BLOCKS && layout != RD_LAYOUT_COMPACT) return rd_fail(RD_ERR_ARG, "unknown layout");
    if (sim->ws) return rd_fail(RD_ERR_STATE, "set the layout before bind");
    if (layout == RD_LAYOUT_COMPACT) {
        if (sim->g->B != 8) return rd_fail(RD_ERR_SHAPE, "the compact layout needs 8^3 blocks");
        // byte offsets of one species buffer (4 bytes per voxel at most) stay 32-bit
        if (sim->g->n_active > (int64_t)(0xFFFFFF00u / 4) - 64)
            return rd_fail(RD_ERR_SHAPE, "the compact layout holds at most 2^30 - 128 active voxels");
        // its kernels take a block's x neighbours as list entries b - 1 and b + 1 (the
        // builder lists blocks x-fastest, and concatenation keeps each part's order)
        const std::vector<BlockInfo> &info = sim->g->info;
        for (size_t b = 0; b < info.size(); ++b)
            if ((info[b].nbr[0] >= 0 && info[b].nbr[0] != (int32_t)b - 1) ||
                (info[b].nbr[1] >= 0 && info[b].nbr[1] != (int32_t)b + 1))
                return rd_fail(RD_ERR_STATE, "the compact layout needs x neighbours at adjacent list entries");
        if (sim->kernel < 2) sim->kernel = 2;
    } else if (sim->kernel == 4) {
        sim->kernel = 2;  // the lane-exchange kernel needs the compact layout
    }
    sim->compact = layout == RD_LAYOUT_COMPACT;
    sim->cbase_host.clear();
    sim->ccode_host.clear();
    sim->invalidate_graphs();
    return RD_OK;
}

extern "C" rd_status rd_sim_set_kernel(rd_sim *sim, int kernel, int wg_per_cu)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (kernel < 0 || kernel > 4) return rd_fail(RD_ERR_ARG, "kernel in 0..4");
    if (!sim->compact && kernel == 4)
        return rd_fail(RD_ERR_STATE, "kernel 4 (lane exchange) runs on the compact layout only");
    if (wg_per_cu < 1 || wg_per_cu > 32) return rd_fail(RD_ERR_ARG, "wg_per_cu in 1..32");
    if (sim->compact && kernel < 2)
        return rd_fail(RD_ERR_STATE, "the compact layout runs the column kernels (2 or 3) only");
    sim->kernel = kernel;
    sim->wg_per_cu = wg_per_cu;
    sim->invalidate_graphs();
    return RD_OK;
}

extern "C" rd_status rd_sim_set_fused_steps(rd_sim *sim, int steps)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (steps < 1 || steps > 256) return rd_fail(RD_ERR_ARG, "steps per launch in 1..256");
    if (steps > 1 && (sim->g->B != 8 || sim->compact))
        return rd_fail(RD_ERR_STATE, "fused steps need 8^3 blocks and the block layout");
    sim->fused_steps = steps;
    sim->invalidate_graphs();
    return RD_OK;
}

extern "C" rd_status rd_sim_get_fused_steps(const rd_sim *sim, int *steps)
{
    if (!sim || !steps) return rd_fail(RD_ERR_ARG, "NULL argument");
    *steps = sim->fused_steps;
    return RD_OK;
}

extern "C" rd_status rd_sim_set_rounding(rd_sim *sim, int stochastic, uint64_t seed)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    sim->sround = stochastic != 0;
    sim->seed = (uint32_t)(seed ^ (seed >> 32));
    sim->invalidate_graphs();
    return RD_OK;
}

extern "C" rd_status rd_sim_workspace_bytes(const rd_sim *sim, uint32_t features,
                                            int64_t checkpoint_slots, size_t *bytes)
{
    if (!sim || !bytes) return rd_fail(RD_ERR_ARG, "NULL argument");
    if (sim->S < 1) return rd_fail(RD_ERR_STATE, "add a species first");
    if (checkpoint_slots < 0) return rd_fail(RD_ERR_ARG, "checkpoint_slots < 0");
    *bytes = sim_layout(*sim, features, checkpoint_slots).total;
    return RD_OK;
}

extern "C" rd_status rd_sim_bind(rd_sim *sim, void *dev_workspace, size_t bytes, uint32_t features,
                                 int64_t checkpoint_slots, void *stream)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (sim->S < 1) return rd_fail(RD_ERR_STATE, "add a species first");
    if (!dev_workspace) return rd_fail(RD_ERR_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)dev_workspace) % 256) return rd_fail(RD_ERR_WORKSPACE, "workspace not 256-byte aligned");
    if (checkpoint_slots < 0) return rd_fail(RD_ERR_ARG, "checkpoint_slots < 0");
    if (sim->compact && (features & (RD_WS_SOLVER | RD_WS_ADJOINT | RD_WS_DIFFUSIVITY)))
        return rd_fail(RD_ERR_STATE, "the compact layout supports stepping, balances, fluxes and region "
                                     "masses; bind the block layout for the solver, adjoint or a factor");
    const SimLayout L = sim_layout(*sim, features, checkpoint_slots);
    if (bytes < L.total)
        return rd_fail(RD_ERR_WORKSPACE, "workspace has " + std::to_string(bytes) + " bytes, needs " +
                                             std::to_string(L.total));
    sim->invalidate_graphs();
    sim->ws = (char *)dev_workspace;
    sim->ws_bytes = bytes;
    sim->L = L;
    sim->features = features;
    sim->diff_on = false;
    sim->band_on = false;  // the upload restores the codes
    sim->e_ones = false;
    sim->cp_slots = checkpoint_slots;
    sim->stream = (hipStream_t)stream;
    return sim->upload();
}

// ---------------------------------------------------------------------------
// rd_sim methods
// ---------------------------------------------------------------------------

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

SimLayout sim_layout(const rd_sim &s, uint32_t features, int64_t cp_slots)
{
    SimLayout L{};
    const rd_geometry &g = *s.g;
    const int64_t nb = g.nb();
    const int64_t NS = (int64_t)g.B * g.B * g.B;
    const size_t es = s.storage == RD_FP32 ? 4 : 2;
    size_t off = 0;
    L.info = off; off = align256(off + sizeof(BlockInfo) * (size_t)std::max<int64_t>(nb, 1));
    L.mask = off; off = align256(off + 8 * (size_t)mask_words(g.B) * (size_t)std::max<int64_t>(nb, 1));
    L.geom = off; off = align256(off + sizeof(GeomInfo) * (size_t)g.nparts());
    if (g.B == 8) {
        L.ncnt = off; off = align256(off + 4 * 64 * (size_t)std::max<int64_t>(nb, 1));
    }
    if (s.compact) {
        // only the active voxels: codes and each species' values in list and slot order
        L.code = off; off = align256(off + (size_t)std::max<int64_t>(g.n_active, 1));
        L.cbase = off; off = align256(off + 4 * (size_t)(nb + 1));
        L.hrec = off; off = align256(off + 4 * 32 * (size_t)std::max<int64_t>(nb, 1));
        L.field_elems = std::max<int64_t>((g.n_active + 63) / 64 * 64, 64);
    } else {
        L.code = off; off = align256(off + (size_t)std::max<int64_t>(nb, 1) * NS);
        L.field_elems = nb * NS;
    }
    for (int p = 0; p < 2; ++p) {
        L.field[p] = off;
        off = align256(off + es * (size_t)L.field_elems * s.S);
    }
    L.nparts = (int)std::max<int64_t>(1, nb);  // one partial row per workgroup (upper bound)
    L.part = off; off = align256(off + sizeof(double) * RD_NRED * (size_t)L.nparts);
    L.mid = off; off = align256(off + sizeof(double) * 16 * RD_FINISH_GROUPS);
    L.res = off; off = align256(off + sizeof(double) * 64);
    if (features & RD_WS_SOLVER) {
        for (int v = 0; v < 4; ++v) {  // r, p, Ap, second p
            L.solver[v] = off;
            off = align256(off + es * (size_t)L.field_elems);
        }
        L.scal = off; off = align256(off + sizeof(double) * 64);
        L.irx = off; off = align256(off + 8 * (size_t)L.field_elems);
    }
    if (features & RD_WS_DIFFUSIVITY) {
        L.diff = off; off = align256(off + 4 * (size_t)std::max<int64_t>(L.field_elems, 1));
        L.diff_stats = off; off = align256(off + 8);
    }
    if (features & RD_WS_ADJOINT) {
        for (int v = 0; v < 2; ++v) {
            L.lam[v] = off;
            off = align256(off + 4 * (size_t)L.field_elems);
        }
        L.target = off; off = align256(off + 4 * (size_t)L.field_elems);
        if (features & RD_WS_DIFFUSIVITY) {
            L.ge = off;
            off = align256(off + 8 * (size_t)std::max<int64_t>(L.field_elems, 1));
        }
        L.cp = off;
        L.cp_stride = align256(es * (size_t)L.field_elems);
        off += L.cp_stride * (size_t)cp_slots;
    }
    L.total = off;
    return L;
}

void rd_sim::invalidate_graphs()
{
    for (auto &e : graphs) hipGraphExecDestroy(e.exec);
    graphs.clear();
}

rd_sim::~rd_sim()
{
    invalidate_graphs();
    if (cap_stream) hipStreamDestroy(cap_stream);
    if (host_res) hipHostFree(host_res);
}

rd_status rd_sim::upload(bool index)
{
    const rd_geometry &G = *g;
    const int64_t nb = G.nb();
    if (index) {
        int dev = 0, ncu = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        if (ncu > 0) n_cu = ncu;
        HIPCHK(hipMemcpyAsync(ws + L.info, G.info.data(), sizeof(BlockInfo) * nb, hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(ws + L.mask, G.mask.data(), 8 * mask_words(G.B) * nb, hipMemcpyHostToDevice,
                              stream));
        if (G.B == 8)
            LAUNCHCHK(rd_launch_count_words8((const uint64_t *)(ws + L.mask), (uint32_t *)(ws + L.ncnt), (int)nb,
                                             stream));
        if (compact) {
            if (cbase_host.size() != (size_t)nb + 1) rd_geometry_compact_index(&G, cbase_host, ccode_host);
            HIPCHK(hipMemcpyAsync(ws + L.code, ccode_host.data(), ccode_host.size(), hipMemcpyHostToDevice,
                                  stream));
            HIPCHK(hipMemcpyAsync(ws + L.cbase, cbase_host.data(), 4 * cbase_host.size(), hipMemcpyHostToDevice,
                                  stream));
            LAUNCHCHK(rd_launch_halo_rec8((const BlockInfo *)(ws + L.info), (const uint64_t *)(ws + L.mask),
                                          (const uint32_t *)(ws + L.cbase), (uint32_t *)(ws + L.hrec), (int)nb,
                                          stream));
        } else {
            HIPCHK(hipMemcpyAsync(ws + L.code, G.code.data(), G.code.size(), hipMemcpyHostToDevice, stream));
        }
        if (G.parts.empty()) geom_host.assign(1, GeomInfo{(int32_t)G.nx, (int32_t)G.ny, (int32_t)G.nz, 0, 0});
        else geom_host = G.parts;
        HIPCHK(hipMemcpyAsync(ws + L.geom, geom_host.data(), sizeof(GeomInfo) * geom_host.size(),
                              hipMemcpyHostToDevice, stream));
    }
    const size_t es = storage == RD_FP32 ? 4 : 2;
    for (int p = 0; p < 2; ++p)
        LAUNCHCHK(rd_launch_fill_u32(ws + L.field[p], 0u, (int64_t)(es * L.field_elems * S / 4), stream));
    // checkpoint / segment slots: the step kernels never write inactive slots, so
    // every buffer they write must start with zeros there
    if (L.cp_stride > 0 && cp_slots > 0)
        LAUNCHCHK(rd_launch_fill_u32(ws + L.cp, 0u, (int64_t)(L.cp_stride * (size_t)cp_slots / 4), stream));
    LAUNCHCHK(rd_launch_fill_u32(ws + L.res, 0u, 64 * 2, stream));  // results + step counter
    if (!host_res) HIPCHK(hipHostMalloc((void **)&host_res, 64 * sizeof(double), hipHostMallocDefault));
    cur = 0;
    steps_taken = 0;
    for (int s = 0; s < S; ++s) {
        rd_status st = apply_dirichlet(s);
        if (st != RD_OK) return st;
    }
    HIPCHK(hipStreamSynchronize(stream));
    return RD_OK;
}

// Write the held Dirichlet values into the current buffer of species s (a scatter
// of the current field through a temporary is avoided: a dedicated pass over the
// blocks sets only the face voxels).
rd_status rd_sim::apply_dirichlet(int s)
{
    if (!ws || !dir[s]) return RD_OK;
    float dv[6];
    for (int f = 0; f < 6; ++f) dv[f] = (float)dirval[s][f];
    LAUNCHCHK(rd_launch_set_dirichlet(storage, g->B, (const BlockInfo *)(ws + L.info),
                                      (const uint64_t *)(ws + L.mask), cbase_ptr(),
                                      (const GeomInfo *)(ws + L.geom), (int)g->nb(), field_ptr(cur, s),
                                      dir[s], dv, stream));
    return RD_OK;
}

void *rd_sim::field_ptr(int buf, int s) const
{
    const size_t es = storage == RD_FP32 ? 4 : 2;
    return ws + L.field[buf] + es * (size_t)L.field_elems * s;
}

StepArgs rd_sim::step_args(double dt, int in_buf) const
{
    StepArgs a{};
    a.info = (const BlockInfo *)(ws + L.info);
    a.mask = (const uint64_t *)(ws + L.mask);
    a.code = (const uint8_t *)(ws + L.code);
    a.ncnt = g->B == 8 ? (const uint32_t *)(ws + L.ncnt) : nullptr;
    a.hrec = compact ? (const uint32_t *)(ws + L.hrec) : nullptr;
    a.cbase = cbase_ptr();
    a.geom = (const GeomInfo *)(ws + L.geom);
    a.cin = field_ptr(in_buf, 0);
    a.cout = field_ptr(1 - in_buf, 0);
    a.sstride = L.field_elems;
    a.nb = (int32_t)g->nb();
    a.S = S;
    a.xcd_chunk = 0;
    const double dx = g->dx;
    for (int s = 0; s < S; ++s) {
        SpeciesCoef &c = a.coef[s];
        double out_rate = 0.0;
        for (const Reaction &r : reactions)
            if (r.from == s) out_rate += r.rate;
        c.alpha = (float)(D[s] * dt / (dx * dx));
        c.beta = (float)(dt * out_rate);
        c.gamma = (float)(robin[s] * dt / dx);
        c.dir = dir[s];
        for (int b = 0; b < RD_MAX_SPECIES; ++b) c.K[b] = 0.0f;
        for (const Reaction &r : reactions)
            if (r.to == s) c.K[r.from] = (float)((double)c.K[r.from] + dt * r.rate);
    }
    return a;
}

double rd_sim::lambda_max() const
{
    const double dx = g->dx;
    double dmax = 0.0, rmax = 0.0, kmax = 0.0;
    for (int s = 0; s < S; ++s) {
        dmax = std::max(dmax, D[s] * (diff_on ? e_max : 1.0));
        kmax = std::max(kmax, robin[s]);
        double out_rate = band_on ? sink[s] : 0.0;
        for (const Reaction &r : reactions)
            if (r.from == s) out_rate += r.rate;
        rmax = std::max(rmax, out_rate);
    }
    return 12.0 * dmax / (dx * dx) + rmax + 6.0 * kmax / dx;
}

rd_status rd_sim::check_dt(double dt) const
{
    if (!(dt > 0.0) || !isfinite(dt)) return rd_fail(RD_ERR_ARG, "dt must be positive");
    const double lm = lambda_max();
    if (lm > 0.0 && dt > 2.0 / lm * (1.0 + 1e-12))
        return rd_fail(RD_ERR_UNSTABLE_DT, "dt = " + std::to_string(dt) + " exceeds 2/lambda_max = " +
                                               std::to_string(2.0 / lm));
    return RD_OK;
}

uint32_t *rd_sim::step_counter() const { return (uint32_t *)(ws + L.res + 384); }

void rd_sim::launch_shape(StepArgs &a) const
{
    a.kernel = g->B == 8 ? kernel : 0;
    a.xcd_chunk = xcd_chunk(a.nb);
    if (a.kernel == 1) {
        // a multiple of 8 (one share per XCD), no more workgroups than blocks need
        int grid = n_cu * wg_per_cu;
        const int need = ((a.nb + 7) / 8) * 8;
        if (grid > need) grid = need;
        a.grid = std::max(8, (grid / 8) * 8);
    }
}

bool rd_sim::fused_ok() const
{
    return g->B == 8 && !compact && (kernel == 2 || kernel == 3) && !diff_path();
}

rd_status rd_sim::launch_steps(double dt, int64_t n)
{
    // stochastic rounding: at the store for 16-bit storage; for FP32 storage a dither of
    // the increment, in the constant-D kernels only (the kernels with a diffusivity
    // factor round FP32 to nearest)
    const bool sr = sround && (storage != RD_FP32 || !diff_path());
    if (fused_steps > 1 && fused_ok()) {
        for (int64_t i = 0; i < n; i += fused_steps) {
            const int m = (int)std::min<int64_t>(fused_steps, n - i);
            StepArgs a = step_args(dt, cur);
            launch_shape(a);
            a.sround = sr ? 1 : 0;
            a.seed = seed;
            a.ctr = step_counter();
            a.ctr_off = (uint32_t)i;
            LAUNCHCHK(rd_launch_step_fused(storage, a, m, n_cu, stream));
            if (m & 1) cur = 1 - cur;
        }
        if (sr && n > 0) LAUNCHCHK(rd_launch_add_u32(step_counter(), (uint32_t)n, stream));
        return RD_OK;
    }
    for (int64_t i = 0; i < n; ++i) {
        StepArgs a = step_args(dt, cur);
        launch_shape(a);
        a.sround = sr ? 1 : 0;
        a.seed = seed;
        a.ctr = step_counter();
        a.ctr_off = (uint32_t)i;
        if (diff_path()) {
            // B = 8: the column kernel (with the x-face exchange when kernel 3 is chosen)
            // unless the workgroup-per-block kernel is chosen (then one thread per slot);
            // B = 4: one thread per slot
            const int column = g->B == 8 && kernel != 0 ? (kernel == 3 ? 2 : 1) : 0;
            const int groups = (a.nb + 3) / 4;
            a.xcd_chunk = column && xcd_map && groups >= 64 ? (groups + 7) / 8 : 0;
            DiffArgs da{a, (const float *)(ws + L.diff), {0.0f, 0.0f, 0.0f, 0.0f}};
            for (int s = 0; s < S; ++s) da.sink[s] = band_on ? (float)(dt * sink[s]) : 0.0f;
            LAUNCHCHK(rd_launch_step_diff(storage, g->B, da, column, stream));
        } else if (compact && kernel == 4) {
            LAUNCHCHK(rd_launch_step_lanes(storage, a, stream));
        } else {
            LAUNCHCHK(rd_launch_step(storage, g->B, a, stream));
        }
        cur = 1 - cur;
    }
    // the device step counter advances once per batch of launches, so graph replay
    // and direct launches see the same counter values
    if (sr && n > 0) LAUNCHCHK(rd_launch_add_u32(step_counter(), (uint32_t)n, stream));
    return RD_OK;
}

int rd_sim::xcd_chunk(int nb) const
{
    if (!xcd_map) return 0;
    // blocks per workgroup: 1 for the B = 8 workgroup kernels, 4 for the wave kernels
    const int bpw = (g->B == 8 && kernel < 2) ? 1 : 4;
    const int groups = (nb + bpw - 1) / bpw;
    if (groups < 64) return 0;
    return (groups + 7) / 8;
}

rd_status rd_sim::step(double dt, int64_t n)
{
    if (!ws) return rd_fail(RD_ERR_STATE, "bind a workspace first");
    if (n < 0) return rd_fail(RD_ERR_ARG, "n_steps < 0");
    rd_status st = check_dt(dt);
    if (st != RD_OK) return st;
    if (n == 0) return RD_OK;
    if (g->nb() == 0) {  // nothing is stored, nothing changes
        steps_taken += n;
        return RD_OK;
    }
    int64_t left = n;
    // a graph holds an even number of steps so the buffer parity it was captured for
    // is the same at every replay (fused steps: cooperative launches, not captured)
    const int gs = graph_steps + (graph_steps & 1);
    if (use_graph && left >= gs && !(fused_steps > 1 && fused_ok())) {
        GraphEntry *ge = nullptr;
        for (auto &e : graphs)
            if (e.dt == dt && e.parity == cur && e.steps == gs) ge = &e;
        if (!ge) {
            if (!cap_stream) HIPCHK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
            hipStream_t user = stream;
            stream = cap_stream;
            const int cur0 = cur;
            HIPCHK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
            rd_status ls = launch_steps(dt, gs);
            hipGraph_t graph = nullptr;
            hipError_t ce = hipStreamEndCapture(cap_stream, &graph);
            stream = user;
            cur = cur0;
            if (ls != RD_OK) {
                if (graph) hipGraphDestroy(graph);
                return ls;
            }
            HIPCHK(ce);
            GraphEntry e{};
            e.dt = dt;
            e.parity = cur0;
            e.steps = gs;
            hipError_t ie = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            HIPCHK(ie);
            graphs.push_back(e);
            ge = &graphs.back();
        }
        while (left >= gs) {
            HIPCHK(hipGraphLaunch(ge->exec, stream));
            left -= gs;
            steps_taken += gs;
        }
    }
    st = launch_steps(dt, left);
    steps_taken += left;
    return st;
}

rd_status rd_sim::balance(int s, double out[RD_NRED], int part)
{
    if (!ws) return rd_fail(RD_ERR_STATE, "bind a workspace first");
    if (s < 0 || s >= S) return rd_fail(RD_ERR_ARG, "bad species");
    if (part >= g->nparts()) return rd_fail(RD_ERR_ARG, "bad part");
    ReduceArgs a{};
    a.info = (const BlockInfo *)(ws + L.info);
    a.mask = (const uint64_t *)(ws + L.mask);
    a.code = (const uint8_t *)(ws + L.code);
    a.cbase = cbase_ptr();
    a.geom = (const GeomInfo *)(ws + L.geom);
    a.c = field_ptr(cur, 0);
    a.sstride = L.field_elems;
    a.b0 = 0;
    a.nb = (int32_t)g->nb();
    if (part >= 0) {
        int64_t first = 0, count = 0;
        rd_geometry_part_info(g, part, nullptr, nullptr, &first, &count);
        a.b0 = (int32_t)first;
        a.nb = (int32_t)count;
    }
    a.S = S;
    a.s = s;
    a.dx = g->dx;
    a.D = D[s];
    a.kR = robin[s];
    a.dir = dir[s];
    for (const Reaction &r : reactions) {
        if (r.from == s) a.rate_out += r.rate;
        if (r.to == s) a.rate_in[r.from] += r.rate;
    }
    a.partial = (double *)(ws + L.part);
    // 0 rows for an empty geometry: sums are 0
    const int nparts = diff_path() ? rd_diff_reduce_rows(g->B, a.nb) : rd_reduce_rows(g->B, a.nb);
    double *res = (double *)(ws + L.res);
    if (diff_path())
        LAUNCHCHK(rd_launch_reduce_diff(storage, g->B, a, (const float *)(ws + L.diff), band_on ? sink[s] : 0.0,
                                        stream));
    else LAUNCHCHK(rd_launch_reduce(storage, g->B, a, stream));
    LAUNCHCHK(rd_launch_finish_reduce(a.partial, nparts, RD_NRED, (double *)(ws + L.mid), res, stream));
    HIPCHK(hipMemcpyAsync(host_res, res, sizeof(double) * RD_NRED, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    for (int l = 0; l < RD_NRED; ++l) out[l] = host_res[l];
    if (out[9] != 0.0) return rd_fail(RD_ERR_NONFINITE, "field holds " + std::to_string((int64_t)out[9]) +
                                                            " non-finite values");
    return RD_OK;
}

// ---------------------------------------------------------------------------
// C ABI wrappers of the methods
// ---------------------------------------------------------------------------

extern "C" rd_status rd_sim_set_field(rd_sim *sim, int species, const float *dev_dense)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (!sim->ws) return rd_fail(RD_ERR_STATE, "bind a workspace first");
    if (species < 0 || species >= sim->S) return rd_fail(RD_ERR_ARG, "bad species");
    if (!dev_dense) return rd_fail(RD_ERR_ARG, "field pointer is NULL");
    float dv[6];
    for (int f = 0; f < 6; ++f) dv[f] = (float)sim->dirval[species][f];
    LAUNCHCHK(rd_launch_scatter(sim->storage, sim->g->B, (const BlockInfo *)(sim->ws + sim->L.info),
                                (const uint64_t *)(sim->ws + sim->L.mask), sim->cbase_ptr(),
                                (const GeomInfo *)(sim->ws + sim->L.geom), (int)sim->g->nb(),
                                dev_dense, sim->field_ptr(sim->cur, species), sim->dir[species], dv,
                                sim->stream));
    sim->steps_taken = 0;
    return RD_OK;
}

// Fill the diffusivity factor (mode 0: values, mode 1: smooth D(phi)), check it and
// switch the steps to the inhomogeneous kernels.
static rd_status set_diffusivity(rd_sim *sim, const float *dev_dense, int mode, double d_min,
                                 double d_max, double g1, double g2)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (!sim->ws) return rd_fail(RD_ERR_STATE, "bind a workspace first");
    if (!(sim->features & RD_WS_DIFFUSIVITY))
        return rd_fail(RD_ERR_WORKSPACE, "bind with RD_WS_DIFFUSIVITY for a diffusivity factor");
    if (!dev_dense && mode != 2) return rd_fail(RD_ERR_ARG, "array pointer is NULL");
    if (mode == 1 && !(std::isfinite(d_min) && std::isfinite(d_max) && std::isfinite(g1) &&
                       std::isfinite(g2) && d_min >= 0.0 && d_max >= 0.0))
        return rd_fail(RD_ERR_ARG, "need finite d_min, d_max >= 0 and finite gamma1, gamma2");
    char *ws = sim->ws;
    const SimLayout &L = sim->L;
    uint32_t *stats = (uint32_t *)(ws + L.diff_stats);
    LAUNCHCHK(rd_launch_set_diff(sim->g->B, (const BlockInfo *)(ws + L.info), (const uint8_t *)(ws + L.code),
                                 (const GeomInfo *)(ws + L.geom), (int)sim->g->nb(), dev_dense, mode, d_min,
                                 d_max, g1, g2, (float *)(ws + L.diff), stats, sim->stream));
    HIPCHK(hipMemcpyAsync(sim->host_res, stats, 8, hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(hipStreamSynchronize(sim->stream));
    uint32_t hs[2];
    memcpy(hs, sim->host_res, 8);
    sim->invalidate_graphs();
    sim->e_ones = mode == 2;
    if (mode == 2) return RD_OK;
    if (hs[0] != 0) {
        sim->diff_on = false;
        if (sim->band_on) set_diffusivity(sim, dev_dense, 2, 0.0, 0.0, 0.0, 0.0);  // back to e = 1
        return rd_fail(RD_ERR_ARG, std::to_string(hs[0]) + " active voxels have a negative or non-finite "
                                   "diffusivity factor (the factor is cleared)");
    }
    float emax;
    memcpy(&emax, &hs[1], 4);
    sim->e_max = (double)emax;
    sim->diff_on = true;
    return RD_OK;
}

extern "C" rd_status rd_sim_set_diffusivity(rd_sim *sim, const float *dev_dense)
{
    if (sim && sim->g->nparts() > 1)
        return rd_fail(RD_ERR_STATE, "rd_sim_set_diffusivity: one geometry per simulation only");
    return set_diffusivity(sim, dev_dense, 0, 0.0, 0.0, 0.0, 0.0);
}

extern "C" rd_status rd_sim_set_diffusivity_sdf(rd_sim *sim, const float *dev_sdf, double d_min, double d_max,
                                                double gamma1, double gamma2)
{
    if (sim && sim->g->nparts() > 1)
        return rd_fail(RD_ERR_STATE, "rd_sim_set_diffusivity_sdf: one geometry per simulation only");
    return set_diffusivity(sim, dev_sdf, 1, d_min, d_max, gamma1, gamma2);
}

extern "C" rd_status rd_sim_clear_diffusivity(rd_sim *sim)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (sim->diff_on) sim->invalidate_graphs();
    sim->diff_on = false;
    // the band's sink still runs through the factor kernels, with e = 1
    if (sim->band_on && !sim->e_ones) return set_diffusivity(sim, nullptr, 2, 0.0, 0.0, 0.0, 0.0);
    return RD_OK;
}

bool rd_sim::sink_active() const
{
    if (!band_on) return false;
    for (int s = 0; s < S; ++s)
        if (sink[s] != 0.0) return true;
    return false;
}

extern "C" rd_status rd_sim_set_sink(rd_sim *sim, int species, double rate)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (species < 0 || species >= sim->S) return rd_fail(RD_ERR_ARG, "bad species");
    if (!(rate >= 0.0) || !std::isfinite(rate)) return rd_fail(RD_ERR_ARG, "sink rate must be finite and >= 0");
    sim->sink[species] = rate;
    sim->invalidate_graphs();
    return RD_OK;
}

extern "C" rd_status rd_sim_set_sink_band(rd_sim *sim, const float *dev_phi, double band, int64_t *n_band)
{
    if (sim && sim->g->nparts() > 1)
        return rd_fail(RD_ERR_STATE, "rd_sim_set_sink_band: one geometry per simulation only");
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (!sim->ws) return rd_fail(RD_ERR_STATE, "bind a workspace first");
    if (!(sim->features & RD_WS_DIFFUSIVITY))
        return rd_fail(RD_ERR_WORKSPACE, "bind with RD_WS_DIFFUSIVITY for a sink band");
    if (!dev_phi) return rd_fail(RD_ERR_ARG, "phi is NULL");
    if (!std::isfinite(band)) return rd_fail(RD_ERR_ARG, "band must be finite");
    char *ws = sim->ws;
    const SimLayout &L = sim->L;
    uint32_t *cnt = (uint32_t *)(ws + L.diff_stats);
    LAUNCHCHK(rd_launch_set_band(sim->g->B, (const BlockInfo *)(ws + L.info), (uint8_t *)(ws + L.code),
                                 (const GeomInfo *)(ws + L.geom), (int)sim->g->nb(), dev_phi, band, cnt,
                                 sim->stream));
    HIPCHK(hipMemcpyAsync(sim->host_res, cnt, 4, hipMemcpyDeviceToHost, sim->stream));
    HIPCHK(hipStreamSynchronize(sim->stream));
    uint32_t n;
    memcpy(&n, sim->host_res, 4);
    sim->invalidate_graphs();
    sim->band_on = n > 0;
    if (n_band) *n_band = (int64_t)n;
    // without a factor the band's sink runs through the factor kernels with e = 1
    if (sim->band_on && !sim->diff_on && !sim->e_ones) return set_diffusivity(sim, nullptr, 2, 0.0, 0.0, 0.0, 0.0);
    return RD_OK;
}

extern "C" rd_status rd_sim_get_field(const rd_sim *sim, int species, float *dev_dense)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (!sim->ws) return rd_fail(RD_ERR_STATE, "bind a workspace first");
    if (species < 0 || species >= sim->S) return rd_fail(RD_ERR_ARG, "bad species");
    if (!dev_dense) return rd_fail(RD_ERR_ARG, "field pointer is NULL");
    const rd_geometry &G = *sim->g;
    LAUNCHCHK(rd_launch_gather(sim->storage, G.B, (const BlockInfo *)(sim->ws + sim->L.info),
                               (const uint64_t *)(sim->ws + sim->L.mask), sim->cbase_ptr(),
                               (const GeomInfo *)(sim->ws + sim->L.geom), (int)G.nb(),
                               sim->field_ptr(sim->cur, species), dev_dense, G.nx * G.ny * G.nz,
                               sim->stream));
    return RD_OK;
}

extern "C" rd_status rd_sim_step(rd_sim *sim, double dt, int64_t n_steps)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    return sim->step(dt, n_steps);
}

extern "C" rd_status rd_sim_steps_taken(const rd_sim *sim, int64_t *n)
{
    if (!sim || !n) return rd_fail(RD_ERR_ARG, "NULL argument");
    *n = sim->steps_taken;
    return RD_OK;
}

extern "C" rd_status rd_sim_balance(rd_sim *sim, int species, double out[9])
{
    if (!sim || !out) return rd_fail(RD_ERR_ARG, "NULL argument");
    double r[RD_NRED];
    rd_status st = sim->balance(species, r);
    for (int l = 0; l < 9; ++l) out[l] = r[l];
    return st;
}

extern "C" rd_status rd_sim_balance_part(rd_sim *sim, int species, int part, double out[9])
{
    if (!sim || !out) return rd_fail(RD_ERR_ARG, "NULL argument");
    if (part < 0) return rd_fail(RD_ERR_ARG, "bad part");
    double r[RD_NRED];
    rd_status st = sim->balance(species, r, part);
    for (int l = 0; l < 9; ++l) out[l] = r[l];
    return st;
}

extern "C" rd_status rd_sim_reduce(rd_sim *sim, int species, double *mass, double *dirichlet_inflow,
                                   double *robin_uptake)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    double r[RD_NRED];
    rd_status st = sim->balance(species, r);
    if (mass) *mass = r[0];
    if (dirichlet_inflow) *dirichlet_inflow = r[1] + r[2] + r[3] + r[4] + r[5] + r[6];
    if (robin_uptake) *robin_uptake = r[7];
    return st;
}

extern "C" rd_status rd_sim_plane_flux(rd_sim *sim, int species, int axis, int64_t i0, double *flux)
{
    if (sim && sim->g->nparts() > 1)
        return rd_fail(RD_ERR_STATE, "rd_sim_plane_flux: one geometry per simulation only");
    if (!sim || !flux) return rd_fail(RD_ERR_ARG, "NULL argument");
    if (!sim->ws) return rd_fail(RD_ERR_STATE, "bind a workspace first");
    if (species < 0 || species >= sim->S) return rd_fail(RD_ERR_ARG, "bad species");
    if (axis < 0 || axis > 2) return rd_fail(RD_ERR_ARG, "axis must be 0, 1 or 2");
    const rd_geometry &G = *sim->g;
    const int64_t n = axis == 0 ? G.nx : axis == 1 ? G.ny : G.nz;
    if (i0 < 0 || i0 + 1 >= n)
        return rd_fail(RD_ERR_ARG, "plane index must satisfy 0 <= i0 < n - 1 along the axis");
    const int nb = (int)G.nb();
    const SimLayout &L = sim->L;
    char *ws = sim->ws;
    double *part = (double *)(ws + L.part);
    double *res = (double *)(ws + L.res) + 32;
    hipStream_t stream = sim->stream;
    if (sim->diff_on) {  // mean face coefficient D (e_p + e_q) / 2
        LAUNCHCHK(rd_launch_plane_flux_diff((int)sim->storage, G.B, (const BlockInfo *)(ws + L.info),
                                            (const uint8_t *)(ws + L.code), sim->field_ptr(sim->cur, species),
                                            (const float *)(ws + L.diff), nb, axis, (int)i0, sim->D[species],
                                            G.dx, part, stream));
        LAUNCHCHK(rd_launch_finish_reduce(part, rd_diff_reduce_rows(G.B, nb), 1, (double *)(ws + L.mid), res,
                                          stream));
    } else {
        LAUNCHCHK(rd_launch_plane_flux((int)sim->storage, G.B, (const BlockInfo *)(ws + L.info),
                                       (const uint8_t *)(ws + L.code), sim->cbase_ptr(),
                                       (const uint64_t *)(ws + L.mask), sim->field_ptr(sim->cur, species), nb,
                                       axis, (int)i0, sim->D[species], G.dx, part, stream));
        LAUNCHCHK(rd_launch_finish_reduce(part, rd_reduce_rows(G.B, nb), 1, (double *)(ws + L.mid), res,
                                          stream));
    }
    double h = 0.0;
    HIPCHK(hipMemcpyAsync(&h, res, sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    *flux = h;
    return RD_OK;
}

extern "C" void rd_sim_destroy(rd_sim *sim) { delete sim; }

// ---------------------------------------------------------------------------
// autotuning
// ---------------------------------------------------------------------------

namespace {

struct LaunchCfg {
    int kernel;
    bool xcd, graph;
    int wg, gsteps;
};

// Mean time per step of `steps` steps with the current launch configuration,
// measured with HIP events on the simulation's stream.
rd_status time_steps(rd_sim *sim, double dt, int64_t steps, double *ms)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    hipError_t er = hipEventCreate(&e1);
    if (er != hipSuccess) {
        hipEventDestroy(e0);
        HIPCHK(er);
    }
    rd_status s = sim->step(dt, std::max<int64_t>(1, steps / 4));  // warm-up + graph capture
    if (s == RD_OK && (er = hipEventRecord(e0, sim->stream)) != hipSuccess) s = rd_fail(RD_ERR_HIP, "event");
    if (s == RD_OK) s = sim->step(dt, steps);
    if (s == RD_OK && (er = hipEventRecord(e1, sim->stream)) != hipSuccess) s = rd_fail(RD_ERR_HIP, "event");
    float msf = 0.0f;
    if (s == RD_OK && (er = hipEventSynchronize(e1)) != hipSuccess) s = rd_fail(RD_ERR_HIP, "event sync");
    if (s == RD_OK && (er = hipEventElapsedTime(&msf, e0, e1)) != hipSuccess) s = rd_fail(RD_ERR_HIP, "elapsed");
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (s == RD_OK) *ms = (double)msf / (double)steps;
    return s;
}

}  // namespace

extern "C" rd_status rd_sim_autotune(rd_sim *sim, double dt, int64_t trial_steps, double *best_ms)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (!sim->ws) return rd_fail(RD_ERR_STATE, "bind a workspace first");
    if (trial_steps < 1) return rd_fail(RD_ERR_ARG, "trial_steps >= 1");
    rd_status s = sim->check_dt(dt);
    if (s != RD_OK) return s;
    std::vector<LaunchCfg> cands;
    const int gs[2] = {16, 64};
    for (int gi = 0; gi < 2; ++gi) {
        if (!sim->compact)  // the compact layout has only the column kernels
            for (int xcd = 0; xcd < 2; ++xcd) cands.push_back({0, xcd != 0, true, 8, gs[gi]});
        if (sim->compact) {
            for (int k = 2; k <= 4; ++k)
                for (int xcd = 0; xcd < 2; ++xcd) cands.push_back({k, xcd != 0, true, 8, gs[gi]});
        } else if (sim->g->B == 8) {
            for (int k = 2; k <= 3; ++k)
                for (int xcd = 0; xcd < 2; ++xcd) cands.push_back({k, xcd != 0, true, 8, gs[gi]});
            for (int wg : {2, 4, 8}) cands.push_back({1, true, true, wg, gs[gi]});
        }
    }
    double best = 1e300;
    LaunchCfg bc = cands[0];
    for (const LaunchCfg &c : cands) {
        sim->kernel = c.kernel;
        sim->xcd_map = c.xcd;
        sim->use_graph = c.graph;
        sim->wg_per_cu = c.wg;
        sim->graph_steps = c.gsteps;
        sim->invalidate_graphs();
        double ms = 0.0;
        if ((s = time_steps(sim, dt, trial_steps, &ms)) != RD_OK) return s;
        if (ms < best) {
            best = ms;
            bc = c;
        }
    }
    sim->kernel = bc.kernel;
    sim->xcd_map = bc.xcd;
    sim->use_graph = bc.graph;
    sim->wg_per_cu = bc.wg;
    sim->graph_steps = bc.gsteps;
    sim->invalidate_graphs();
    if (best_ms) *best_ms = best;
    // the trials advanced the fields: start again from zero + Dirichlet values
    return sim->upload(false);  // reset the fields, keep the index and any band marks
}

namespace {
// Key of an autotuning result: the GPU (architecture name and compute-unit count), the
// storage type, species, reactions and Robin walls, and the geometry (extents, block edge,
// every activity mask word), folded with FNV-1a 64.
uint64_t tune_key(const rd_sim *sim)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) {
            h ^= c[i];
            h *= 1099511628211ull;
        }
    };
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        mix(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
        mix(&prop.multiProcessorCount, sizeof(prop.multiProcessorCount));
    }
    const rd_geometry &g = *sim->g;
    const int64_t dims[5] = {g.nx, g.ny, g.nz, (int64_t)g.B, g.nb()};
    mix(dims, sizeof(dims));
    const int meta[4] = {(int)sim->storage, sim->S, (int)sim->reactions.size(), sim->compact ? 1 : 0};
    mix(meta, sizeof(meta));
    for (int s = 0; s < sim->S; ++s) {
        const int robin = sim->robin[s] != 0.0;
        mix(&robin, sizeof(robin));
    }
    if (!g.mask.empty()) mix(g.mask.data(), g.mask.size() * sizeof(uint64_t));
    return h;
}
}  // namespace

extern "C" rd_status rd_sim_autotune_cached(rd_sim *sim, double dt, int64_t trial_steps, const char *cache_path,
                                            int *from_cache, double *best_ms)
{
    if (!sim || !cache_path) return rd_fail(RD_ERR_ARG, "NULL argument");
    if (!sim->ws) return rd_fail(RD_ERR_STATE, "bind a workspace first");
    const uint64_t key = tune_key(sim);
    char want[32];
    snprintf(want, sizeof(want), "%016llx", (unsigned long long)key);
    // the last entry with this key wins
    bool found = false;
    LaunchCfg c{};
    double ms = 0.0;
    if (FILE *f = fopen(cache_path, "r")) {
        char line[256];
        while (fgets(line, sizeof(line), f)) {
            char tag[16], k[32];
            int kernel, xcd, graph, wg, gsteps;
            double m;
            if (sscanf(line, "%15s %31s %d %d %d %d %d %lf", tag, k, &kernel, &xcd, &graph, &wg, &gsteps, &m) == 8 &&
                strcmp(tag, "rdtune1") == 0 && strcmp(k, want) == 0 && kernel >= 0 && kernel <= 4 && wg >= 1 &&
                gsteps >= 1 && !(sim->g->B == 4 && kernel != 0) && !(sim->compact && kernel < 2) &&
                !(!sim->compact && kernel == 4)) {
                c = {kernel, xcd != 0, graph != 0, wg, gsteps};
                ms = m;
                found = true;
            }
        }
        fclose(f);
    }
    if (found) {
        sim->kernel = c.kernel;
        sim->xcd_map = c.xcd;
        sim->use_graph = c.graph;
        sim->wg_per_cu = c.wg;
        sim->graph_steps = c.gsteps;
        sim->invalidate_graphs();
        if (from_cache) *from_cache = 1;
        if (best_ms) *best_ms = ms;
        return RD_OK;
    }
    rd_status s = rd_sim_autotune(sim, dt, trial_steps, &ms);
    if (s != RD_OK) return s;
    FILE *f = fopen(cache_path, "a");
    if (!f) return rd_fail(RD_ERR_ARG, std::string("cannot append to the autotuning cache ") + cache_path);
    const int ok = fprintf(f, "rdtune1 %s %d %d %d %d %d %.9g\n", want, sim->kernel, sim->xcd_map ? 1 : 0,
                           sim->use_graph ? 1 : 0, sim->wg_per_cu, sim->graph_steps, ms);
    if (fclose(f) != 0 || ok < 0)
        return rd_fail(RD_ERR_ARG, std::string("cannot write the autotuning cache ") + cache_path);
    if (from_cache) *from_cache = 0;
    if (best_ms) *best_ms = ms;
    return RD_OK;
}

extern "C" rd_status rd_autotune_pick(rd_sim *const *sims, int n, double dt, int64_t trial_steps,
                                      int *best_index, double *ms_per_step)
{
    if (!sims || n <= 0 || !best_index) return rd_fail(RD_ERR_ARG, "need sims and best_index");
    double best = 1e300;
    *best_index = -1;
    for (int i = 0; i < n; ++i) {
        double ms = 0.0;
        rd_status s = rd_sim_autotune(sims[i], dt, trial_steps, &ms);
        if (s != RD_OK) return s;
        if (ms_per_step) ms_per_step[i] = ms;
        if (ms < best) {
            best = ms;
            *best_index = i;
        }
    }
    return RD_OK;
}

extern "C" rd_status rd_sim_get_launch(const rd_sim *sim, int *graph_steps, int *use_graph,
                                       int *xcd_map, int *kernel, int *wg_per_cu)
{
    if (!sim) return rd_fail(RD_ERR_ARG, "sim is NULL");
    if (graph_steps) *graph_steps = sim->graph_steps;
    if (use_graph) *use_graph = sim->use_graph;
    if (xcd_map) *xcd_map = sim->xcd_map;
    if (kernel) *kernel = sim->kernel;
    if (wg_per_cu) *wg_per_cu = sim->wg_per_cu;
    return RD_OK;
}
