// rd_diff.h -- inhomogeneous diffusion: a per-slot diffusivity factor e.
//
// Species s diffuses with D_s(x) = D_s * e(x); the coefficient of the face between
// voxels p and q is the arithmetic mean D_s (e_p + e_q) / 2, and faces toward
// inactive voxels carry no flux (mirror rule), as in the inhomogeneous-diffusion
// functor of the paper's appendix "Code examples".  e is FP32, block-major like the
// fields (nb * B^3 slots), 0 on inactive slots.
//
// The same kernels apply a volumetric sink on a near-surface band (paper: section
// "Application example 2", a sink restricted to the surface by the level set): bit 7 of
// a slot's code byte marks the band, and species s loses dt k_s c there each step.
#define RD_CODE_BAND 0x80u
#pragma once

#include "rd_internal.h"

struct DiffArgs {
    StepArgs s;       // the step's own arguments (coef[].alpha = D_s dt / dx^2)
    const float *e;   // diffusivity factor per slot
    float sink[RD_MAX_SPECIES];  // dt * k_s, applied on band slots
};

// One step with the factor.  column = 1 (B = 8 only): one wave per block walking
// z-columns; column = 2: the same with the x faces of x-adjacent blocks of a workgroup
// handed over through LDS; column = 0: one thread per slot.  All give the same bits.
int rd_launch_step_diff(int storage, int B, const DiffArgs &a, int column, void *stream);

// Fill e from a dense float32 (nz, ny, nx) device array: mode 0 copies the values,
// mode 1 maps a signed distance phi to d_min + d_max / (1 + exp(-(g1 + g2 phi))),
// mode 2 sets 1 on every active slot (dense is not read).
// stats (two uint32 words, cleared here) receive the number of active slots whose
// value is negative or not finite, and the bit pattern of the largest value.
int rd_launch_set_diff(int B, const BlockInfo *info, const uint8_t *code, const GeomInfo *geom,
                       int nb, const float *dense, int mode, double d_min, double d_max, double g1,
                       double g2, float *e, uint32_t *stats, void *stream);

// Balance terms (the lanes of the homogeneous reduction) with the factor: the
// Dirichlet inflow of a face uses the mean coefficient.  Writes rd_diff_reduce_rows
// rows of RD_NRED partials.
int rd_diff_reduce_rows(int B, int nb);
// ksink: the reduced species' sink rate k_s (its band term goes to the uptake lane).
int rd_launch_reduce_diff(int storage, int B, const ReduceArgs &a, const float *e, double ksink,
                          void *stream);

// One FP64 partial per rd_diff_reduce_rows row: D sum over active pairs straddling the
// plane i0 | i0 + 1 along axis of (e_p + e_q) / 2 (c_p - c_q) dx.
int rd_launch_plane_flux_diff(int storage, int B, const BlockInfo *info, const uint8_t *code, const void *c,
                              const float *e, int nb, int axis, int i0, double D, double dx, double *partial,
                              void *stream);

// Mark the band: bit 7 of the code byte of active slots set where phi < band, cleared
// elsewhere; count (one uint32, cleared here) receives the number of band slots.
int rd_launch_set_band(int B, const BlockInfo *info, uint8_t *code, const GeomInfo *geom, int nb,
                       const float *phi, double band, uint32_t *count, void *stream);
