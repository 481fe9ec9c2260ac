// rd_adjoint.h -- arguments of the adjoint kernels.
#pragma once

#include <stdint.h>

#include "rd_internal.h"

struct AdjArgs {
    const BlockInfo *info;
    const uint64_t *mask;
    const GeomInfo *geom;
    int nb;
    SpeciesCoef coef;     // forward coefficients of the species (K unused)
    const float *lam_in;  // lambda^{n+1}, FP32 block-major
    float *lam_out;       // lambda^n
    const void *c;        // c^n in the storage type
    const float *seed;    // seed field (block-major FP32)
    double *partial;      // per-workgroup partials
};

int adj_groups(int B, int nb);
int adj_launch_step(int storage, int B, const AdjArgs &a, void *stream);
int adj_launch_seed(int storage, int B, const AdjArgs &a, int mode, void *stream);
int adj_launch_sum_acc(const double *part, int nparts, int nl, double *out, void *stream);
