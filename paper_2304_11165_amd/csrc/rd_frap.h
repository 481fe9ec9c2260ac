// rd_frap.h -- region mass (the bleached box of a simulated FRAP experiment).
#pragma once

#include "rd_internal.h"

// FP64 sum of field c of one species over the active voxels with x0 <= gx < x1,
// y0 <= gy < y1, z0 <= gz < z1 (region = {x0, x1, y0, y1, z0, z1}), one partial per
// workgroup: rd_region_rows(B, nb) rows of one double.
int rd_region_rows(int B, int nb);
int rd_launch_region_mass(int storage, int B, const BlockInfo *info, const uint8_t *code, const uint32_t *cbase,
                          const uint64_t *mask, const void *c,
                          int nb, const int32_t region[6], double *partial, void *stream);
