// rd_solve.h -- conjugate-gradient steady state (single geometry or batch).
#pragma once

#include <stdint.h>

#include "rd_internal.h"

// per-geometry scalar slots (doubles) in CgArgs::scal
enum {
    CG_ALPHA = 0,
    CG_BETA = 1,
    CG_RR = 2,
    CG_PAP = 3,
    CG_BB = 4,
    CG_RRNEW = 5,
    CG_DONE = 6,
    CG_CHECK = 7,
    CG_QIN = 8,
    CG_QOUT = 9,
    CG_SIGMA = 10,       // FP64 iterate: r and p hold sigma times the true residual / direction
    CG_SIGMA_PREV = 11,  // the scale r and p hold before a pending rescaling (powers of 2)
    CG_RRREC = 12,       // r.r of the recursive residual (CG_RR / CG_RRNEW hold r.z: with the
                         // preconditioner z = M^-1 r, without it z = r)
    CG_REPL = 13,        // at a check: 2 replace the residual, 3 only rescale, 0 leave it
    CG_NSCAL = 14
};

struct CgArgs {
    const BlockInfo *info;
    const uint64_t *mask;
    const uint8_t *code;   // per-slot neighbour codes (bits 0-5 neighbours, bit 6 active)
    const GeomInfo *geom;  // ngeom entries; block ranges via block0
    int nb;
    int ngeom;
    uint32_t dir;          // Dirichlet faces (inlet | outlet)
    void *x, *r, *p, *ap;  // storage type T, nb * B^3 each (ap: B = 4 only)
    double *x64;           // FP64 iterate
    int x64_direct;        // with x64: 1 = every update goes to x64 (16 bytes per voxel);
                           // 0 = x accumulates the updates and is folded into x64 at
                           // every check (the iterate is x64 + x / sigma)
    void *p2;              // second p buffer (B = 8: the fused p update writes here)
    double *partial;       // [nb][2]
    double *scal;          // [ngeom][CG_NSCAL]
    double *mid;           // single geometry: scratch of >= 1040 doubles for two-level sums
                           // of long block lists (NULL: one workgroup per geometry)
    void *z;               // B = 8 with prec > 0: the preconditioned residual z = M^-1 r
    int prec;              // B = 8: Jacobi steps of the block preconditioner (0: plain CG)
};

int cg_launch_matvec(int storage, int B, const CgArgs &a, void *stream);
// B = 8: p2 = z + beta p (per live geometry, rounded to the storage type; z = r when
// a.prec is 0) and the partial (p2.A p2, 0); A p2 is not stored.  The caller then swaps
// p and p2.
int cg_launch_matvec_fused(int storage, const CgArgs &a, void *stream);
// x += alpha p, r -= alpha A p, partial (r.z, r.r); B = 4 reads the stored A p, B = 8
// recomputes it from p and, with a.prec > 0, also writes z = M^-1 r.
int cg_launch_update(int storage, int B, const CgArgs &a, void *stream);
// B = 8, a.prec > 0: z = M^-1 r of the stored r on live geometries, partial (r.z, r.r)
int cg_launch_prec(int storage, const CgArgs &a, void *stream);
int cg_launch_pupdate(int storage, int B, const CgArgs &a, void *stream);
// per-block FP64 partials (inlet, outlet) of the flux of x64 through the Dirichlet planes
int cg_launch_flux(int B, const CgArgs &a, int inlet_face, void *stream);
int cg_launch_segsum(const CgArgs &a, int slot0, int slot1, int mode, void *stream);
// Initial guess of the unit-drop problem along `axis` into a.x (every slot, rounded to
// the storage type) and a.x64 (FP64), from the
// 6-connected clusters of active voxels labelled on the GPU.  Scratch: par[nslots]
// (uint32), flags[2 * nslots] (bytes, zeroed by the caller), perc[ngeom] (uint32,
// zeroed by the caller; set to 1 for geometries with a cluster touching both planes).
// FP64 iterate helpers: rows of 256 slots; x = X rounded to the storage type.
int ir_rows(int64_t nslots);
// r = b - A x64 in FP64 (per-block partials (r.r, b.b)); store 1 writes it to r and p;
// store 2 writes sigma r to r and rescales p; store 3 only rescales r and p.  B = 8 with
// store 0 (the check) evaluates the unfolded iterate x64 + x / sigma when x64_direct is 0.
int cg_launch_res64(int storage, int B, const CgArgs &a, int store, void *stream);
int ir_launch_store(int storage, int64_t nslots, const double *X, void *x, void *stream);
// x64 += x / sigma (per geometry), x = 0
int ir_launch_fold(int storage, int B, const CgArgs &a, int64_t nslots, void *stream);
int cg_launch_initial_guess(int storage, int B, const CgArgs &a, int axis, int64_t nslots, uint32_t *par,
                            uint8_t *flags, uint32_t *perc, void *stream);
