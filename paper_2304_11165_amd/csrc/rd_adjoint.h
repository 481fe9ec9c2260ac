// rd_adjoint.h -- arguments of the adjoint kernels.
#pragma once

#include <stdint.h>

#include "rd_internal.h"

struct AdjArgs {
    const BlockInfo *info;
    const uint64_t *mask;
    const uint8_t *code;  // per-slot neighbour codes (bits 0-5 neighbours, bit 6 active)
    const GeomInfo *geom;
    int nb;
    SpeciesCoef coef;     // forward coefficients of the species (K unused)
    const float *lam_in;  // lambda^{n+1}, FP32 block-major
    float *lam_out;       // lambda^n
    const void *c;        // c^n in the storage type
    const float *seed;    // seed field (block-major FP32)
    double *partial;      // step: per-block (B = 8) or per-workgroup (B = 4) FP64 gradient
                          // accumulators [parts][2], added to in step order; seed: [nb]
};

// The adjoint step with a per-slot diffusivity factor e (face coefficient
// (e_p + e_q) / 2): lambda^n from lambda^{n+1}, the dL/dD and dL/dk rows as above, and
// dL/de_p += alpha / 2 * sum_{q active nb} (c_q - c_p)(lambda_p - lambda_q) per slot (FP64,
// ge, added to in step order).  column = 1 (B = 8): one wave per block walking
// z-columns; otherwise one thread per slot.  Rows: one per block for B = 8.
struct AdjEArgs {
    AdjArgs a;
    const float *e;
    double alpha;  // D dt / dx^2 in FP64
    double *ge;    // dL/de per slot
};
int adj_launch_step_e(int storage, int B, const AdjEArgs &x, int column, void *stream);
// dense (nz, ny, nx) FP64 copy of a per-slot FP64 array (0 off the active voxels)
int adj_launch_dense_f64(int B, const BlockInfo *info, const uint8_t *code, const GeomInfo *geom, int nb,
                         const double *v, double *dense, int64_t ndense, void *stream);

// gradient accumulator rows of the step kernel (B = 8: one per block; B = 4: one per
// workgroup of four blocks)
int adj_groups(int B, int nb);
int adj_launch_step(int storage, int B, const AdjArgs &a, void *stream);
int adj_launch_seed(int storage, int B, const AdjArgs &a, int mode, void *stream);
