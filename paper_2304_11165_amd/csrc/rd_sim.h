// rd_sim.h -- the simulation handle behind rd_sim*.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "rd_host.h"

#include <string>

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return rd_fail(RD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)
#define LAUNCHCHK(expr)                                                                      \
    do {                                                                                     \
        int e_ = (expr);                                                                     \
        if (e_ != 0)                                                                         \
            return rd_fail(RD_ERR_HIP, std::string(#expr) + ": " +                           \
                                           hipGetErrorString((hipError_t)e_));               \
    } while (0)

struct Reaction {
    int from, to;
    double rate;
};

// Byte offsets of every array inside the caller's workspace.
struct SimLayout {
    size_t info, mask, geom, code;
    size_t cbase;         // compact layout: first voxel of each block, uint32[nb + 1]
    size_t ncnt;          // B = 8: active-neighbour counts, uint32[nb][64] (3 bits per plane)
    size_t hrec;          // compact layout: halo records, uint32[nb][32]
    size_t field[2];
    int64_t field_elems;  // nb * B^3
    int nparts;
    size_t part, mid, res;  // reduction partials, finish scratch, results
    size_t solver[4], scal;  // CG vectors r, p, Ap, second p
    size_t irx;              // FP64 iterate of the steady state
    size_t diff, diff_stats; // per-slot diffusivity factor (FP32) and its set-up counters
    size_t lam[2], target, cp, cp_stride;
    size_t ge;               // dL/de per slot (FP64), adjoint with a diffusivity factor
    size_t total;
};

struct GraphEntry {
    double dt;
    int parity;
    int steps;
    hipGraphExec_t exec;
};

SimLayout sim_layout(const struct rd_sim &s, uint32_t features, int64_t cp_slots);

struct rd_sim {
    const rd_geometry *g = nullptr;
    rd_storage storage = RD_FP32;
    int S = 0;
    double D[RD_MAX_SPECIES] = {0, 0, 0, 0};
    double robin[RD_MAX_SPECIES] = {0, 0, 0, 0};
    uint32_t dir[RD_MAX_SPECIES] = {0, 0, 0, 0};
    double dirval[RD_MAX_SPECIES][6] = {};
    std::vector<Reaction> reactions;

    int graph_steps = 32;
    bool use_graph = true;
    bool xcd_map = true;
    int cg_prec = 6;  // steady-state CG: Jacobi steps of the block preconditioner (0: none)
    int kernel = 2;       // B = 8 step kernel: 0 workgroup per block, 1 persistent, 2 z-column,
                          // 3 z-column with in-workgroup x-face exchange
    int wg_per_cu = 8;    // resident workgroups per CU of the persistent grid
    int n_cu = 256;       // compute units of the bound device
    bool sround = false;  // stochastic rounding on store (BF16 / FP16 storage)
    bool compact = false; // fields hold only the active voxels (B = 8; rd_sim_set_layout)
    int fused_steps = 1;  // steps per cooperative launch (rd_sim_set_fused_steps; 1: off)
    // the fused launch applies: B = 8, block layout, a column kernel, constant D
    bool fused_ok() const;
    std::vector<uint32_t> cbase_host;  // compact index, built at bind
    std::vector<uint8_t> ccode_host;
    uint32_t seed = 0;
    bool diff_on = false;  // a diffusivity factor is set (inhomogeneous diffusion)
    double e_max = 0.0;    // its largest value over the active voxels
    double sink[RD_MAX_SPECIES] = {0, 0, 0, 0};  // volumetric sink rate on the band
    bool band_on = false;  // band slots are marked (code bit 7)
    bool e_ones = false;   // the factor buffer holds 1 on active slots (band without factor)
    bool sink_active() const;
    bool diff_path() const { return diff_on || sink_active(); }

    char *ws = nullptr;
    size_t ws_bytes = 0;
    uint32_t features = 0;
    int64_t cp_slots = 0;
    SimLayout L{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<GeomInfo> geom_host;  // one entry per part (the device copy's source)
    double *host_res = nullptr;  // pinned
    std::vector<GraphEntry> graphs;

    int cur = 0;  // buffer holding the current field
    int64_t steps_taken = 0;

    ~rd_sim();
    void invalidate_graphs();
    // index = true: copy the block index, masks and codes too (bind); false: only reset
    // the fields and counters (the codes keep any sink-band marks)
    rd_status upload(bool index = true);
    rd_status apply_dirichlet(int s);
    void *field_ptr(int buf, int s) const;
    const uint32_t *cbase_ptr() const { return compact ? (const uint32_t *)(ws + L.cbase) : nullptr; }
    StepArgs step_args(double dt, int in_buf) const;
    double lambda_max() const;
    rd_status check_dt(double dt) const;
    int xcd_chunk(int nb) const;
    uint32_t *step_counter() const;
    void launch_shape(StepArgs &a) const;
    rd_status launch_steps(double dt, int64_t n);
    rd_status step(double dt, int64_t n);
    // part < 0: every block; else the blocks of one part of a concatenated geometry
    rd_status balance(int s, double out[RD_NRED], int part = -1);
};

int rd_launch_set_dirichlet(int storage, int B, const BlockInfo *info, const uint64_t *mask,
                            const uint32_t *cbase, const GeomInfo *geom, int nb, void *field, uint32_t dir,
                            const float dv[6], void *stream);
