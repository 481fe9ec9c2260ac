// rd_internal.h -- structures shared by the host runtime and the HIP kernels.
//
// Device layout of a bound simulation (all inside the caller's workspace):
//   info   BlockInfo[nb]            neighbour list indices + block position
//   mask   uint64[nb * MW(B)]       own active bits, then face bits of the neighbours
//   fields T[2][S][nb][B^3]         ping-pong buffers, block-major, slot (lz*B+ly)*B+lx;
//                                   compact layout (B = 8): T[2][S][n_active'] holding
//                                   only the active voxels, block by block in slot
//                                   order, block b starting at cbase[b]
//   part   double[...]              per-workgroup FP64 partials of reductions
//   res    double[32]               reduction results
//   (+ solver / adjoint vectors when requested)
#pragma once

#include <stdint.h>

#define RD_MAX_SPECIES 4
#define RD_NRED 10  // reduction lanes: mass, inflow[6], uptake, react, nonfinite count

// 32-byte block record.  nbr: list index of the -x,+x,-y,+y,-z,+z neighbour or -1.
// xy = bx | (by << 16); zg = bz | (geometry id << 16) (the id is 0 outside batches).
struct BlockInfo {
    int32_t nbr[6];
    int32_t xy;
    int32_t zg;
};

// Mask record (uint64 words per block).
//  B = 8: words 0..7 own bits (word lz holds bit ly*8+lx), words 8..13 face bits of the
//         six neighbours (f = 0..5), words 14..15 the active slots below each plane
//         (16 bits per plane z, at bit 16 (z % 4) of word 14 + z / 4).
//  B = 4: word 0 own bits (bit (lz*4+ly)*4+lx); word 1 faces 0..3 (16 bits each, face f
//         at bit 16*f); word 2 faces 4..5 (face 4 at bit 0, face 5 at bit 16).
// Face bit index of face f: x faces (f=0,1): lz*B+ly; y faces: lz*B+lx; z faces: ly*B+lx.
// It is the active bit of the neighbour voxel across that face (0 if no neighbour block).
constexpr int mask_words(int B) { return B == 8 ? 16 : 3; }

// Per-species coefficients of one FTCS step (FP32, computed on the host in FP64).
struct SpeciesCoef {
    float alpha;   // D dt / dx^2
    float beta;    // dt * sum of first-order rates out of the species
    float gamma;   // k_R dt / dx
    uint32_t dir;  // bit f set: face f is Dirichlet
    float K[RD_MAX_SPECIES];  // dt * rate of (b -> this species), indexed by b
};

// Per-geometry data (single geometry: one entry).
struct GeomInfo {
    int32_t nx, ny, nz;
    int32_t block0;  // first list index of this geometry
    int64_t dense0;  // first element of this geometry's box in a dense array holding the
                     // boxes of several geometries one after another (0 for one geometry)
};

struct StepArgs {
    const BlockInfo *info;
    const uint64_t *mask;
    const uint8_t *code;   // per-slot neighbour codes (bits 0-5 neighbours, bit 6 active)
    const uint32_t *hrec;  // compact layout: per-block halo record, 32 words (k_halo_rec8)
    const uint32_t *ncnt;  // B = 8: active-neighbour counts, one word per (block, lane
                           // (x, y)): bits 3z..3z+2 hold the count of voxel (x, y, z)
    const uint32_t *cbase; // compact layout: first voxel of each block (nb + 1); NULL:
                           // block-major layout with every slot stored
    const GeomInfo *geom;  // indexed by geometry id
    const void *cin;       // T*, species-major
    void *cout;
    int64_t sstride;       // elements between species buffers (nb * B^3)
    int32_t nb;            // blocks in the list
    int32_t S;             // species
    int32_t xcd_chunk;     // blocks per XCD chunk in the XCD-aware mapping (0 = plain)
    int32_t kernel;        // B = 8: 0 one workgroup per block, 1 persistent prefetching
                           // kernel with `grid` workgroups, 2 one wave per block (z-columns),
                           // 3 as 2 with x faces exchanged inside the workgroup
    int32_t grid;
    // stochastic rounding on store (BF16 / FP16 storage): the random bits of a slot
    // are hash(slot, species, step, seed) with step = *ctr + ctr_off
    int32_t sround;
    uint32_t seed;
    uint32_t ctr_off;
    const uint32_t *ctr;
    SpeciesCoef coef[RD_MAX_SPECIES];
};

struct ReduceArgs {
    const BlockInfo *info;
    const uint64_t *mask;
    const uint8_t *code;  // per-slot neighbour codes (as in StepArgs)
    const uint32_t *cbase;  // compact layout (as in StepArgs) or NULL
    const GeomInfo *geom;
    const void *c;      // T*
    int64_t sstride;
    int32_t b0;         // first block of the reduced range (list index)
    int32_t nb;         // blocks in the range
    int32_t S;
    int32_t s;          // species reduced
    double dx;
    double D;           // diffusion coefficient of species s
    double kR;          // Robin coefficient of s
    double rate_out;    // sum of rates out of s
    double rate_in[RD_MAX_SPECIES];
    uint32_t dir;       // Dirichlet faces of s
    double *partial;    // [gridDim][RD_NRED]
};

// ---- launchers (k_step.hip) -------------------------------------------------
// storage: 0 fp32, 1 bf16, 2 fp16.  All return a hipError_t as int.
int rd_launch_step(int storage, int B, const StepArgs &a, void *stream);
// Compact layout, B = 8: the column step with lane-exchanged neighbours (k_compact.hip).
int rd_launch_step_lanes(int storage, const StepArgs &a, void *stream);
// rows of partials written by rd_launch_reduce (one per workgroup of four blocks)
int rd_reduce_rows(int B, int nb);
int rd_launch_reduce(int storage, int B, const ReduceArgs &a, void *stream);
// one FP64 partial per rd_reduce_rows row: flux of field c through plane i0 | i0 + 1
int rd_launch_plane_flux(int storage, int B, const BlockInfo *info, const uint8_t *code,
                         const uint32_t *cbase, const uint64_t *mask, const void *c, int nb, int axis,
                         int i0, double D, double dx, double *partial, void *stream);
// Fixed-order sums of partial[nparts][nlanes] (nlanes <= 16) into out[nlanes]; mid is
// scratch of RD_FINISH_GROUPS * nlanes doubles.
#define RD_FINISH_GROUPS 256
int rd_launch_finish_reduce(const double *partial, int nparts, int nlanes, double *mid, double *out,
                            void *stream);
// cbase: compact layout (B = 8) or NULL (block-major), as in StepArgs
int rd_launch_scatter(int storage, int B, const BlockInfo *info, const uint64_t *mask,
                      const uint32_t *cbase, const GeomInfo *geom, int nb, const float *dense, void *field,
                      uint32_t dir, float dir_value_per_face[6], void *stream);
int rd_launch_gather(int storage, int B, const BlockInfo *info, const uint64_t *mask,
                     const uint32_t *cbase, const GeomInfo *geom, int nb, const void *field, float *dense,
                     int64_t ndense, void *stream);
int rd_launch_fill_u32(void *ptr, uint32_t value, int64_t n_words, void *stream);
// B = 8, block layout, column kernels (a.kernel 2 or 3): nsteps steps in one cooperative
// launch (grid barrier between steps); the buffers swap after each step, as in nsteps
// single-step launches; a.ctr_off is the first step's offset.  n_cu: compute units.
int rd_launch_step_fused(int storage, const StepArgs &a, int nsteps, int n_cu, void *stream);
// compact layout: the halo records (StepArgs::hrec) of nb blocks
int rd_launch_halo_rec8(const BlockInfo *info, const uint64_t *mask, const uint32_t *cbase, uint32_t *hrec,
                        int nb, void *stream);
// B = 8: the active-neighbour count words (StepArgs::ncnt) of nb blocks
int rd_launch_count_words8(const uint64_t *mask, uint32_t *ncnt, int nb, void *stream);
int rd_launch_add_u32(uint32_t *ptr, uint32_t add, void *stream);
