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

// gradient accumulator rows of the step kernel (B = 8: one per block; B = 4: one per
// workgroup of four blocks)
int adj_groups(int B, int nb);
int adj_launch_step(int storage, int B, const AdjArgs &a, void *stream);
int adj_launch_seed(int storage, int B, const AdjArgs &a, int mode, void *stream);
