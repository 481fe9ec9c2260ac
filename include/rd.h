/*
 * rd.h -- C ABI of the MI355X sparse-block reaction-diffusion library (librd.so).
 *
 * The library advances reaction-diffusion fields by explicit FTCS time stepping
 * on a sparse block grid fitted to a porous geometry: Stark & Sbalzarini, "An
 * open-source pipeline for solving continuous reaction-diffusion models in
 * image-based geometries of porous media" (arXiv 2304.11165).
 *
 *   PDE        du/dt = div(D grad u) + f(u)               section "Methods", eq. reaction_diffusion
 *   scheme     forward Euler + centred 7-point differences section "Discretization and numerical methods"
 *   walls      no-flux by the mirror rule inside the stencil (same section; appendix "Code examples")
 *   storage    only blocks of B^3 voxels that hold an active voxel are stored
 *              (section "Parallel implementation using OpenFPM")
 *
 * Per free active voxel p and species a, one step computes
 *   c'_a(p) = c_a(p) + alpha_a * sum_{q in N6(p), q active} (c_a(q) - c_a(p))
 *             - (beta_a + gamma_a * n_wall(p)) * c_a(p) + sum_b K_ab * c_b(p)
 * with alpha_a = D_a dt/dx^2, gamma_a = k_R,a dt/dx (Robin wall uptake per wall
 * face), beta_a = dt * (sum of first-order rates out of a), K_ab = dt * (rate of
 * b -> a).  n_wall(p) counts in-box face neighbours that are not active; box
 * faces are no-flux and not walls.  Dirichlet voxels (the active voxels of a box
 * face plane flagged for a species) hold their value and act as active
 * neighbours.
 *
 * Conventions
 *   - Volumes are C-ordered (nz, ny, nx), x fastest.  Voxel (i,j,k) sits at
 *     (i,j,k)*dx.  Face ids: 0:-x 1:+x 2:-y 3:+y 4:-z 5:+z.
 *   - Host pointers are read only during the call.  Device pointers are
 *     caller-owned (for example torch tensors); the library never frees them.
 *   - All device work of a simulation is enqueued on the stream given to
 *     rd_sim_bind (a hipStream_t passed as void*; NULL = the null stream).
 *     rd_sim_step is asynchronous; functions that return host values
 *     synchronise that stream.
 *   - Every function returns rd_status; no C++ exception crosses the ABI.  After
 *     a failure rd_last_error() gives a thread-local message.
 *   - A handle must not be used from two threads at once.
 */
#ifndef RD_H
#define RD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RD_OK = 0,
    RD_ERR_ARG = 1,               /* bad argument value (id, face, pointer, ...) */
    RD_ERR_SHAPE = 2,             /* bad volume shape or block edge */
    RD_ERR_INCONSISTENT_SDF = 3,  /* sign(sdf) > 0 disagrees with image != 0 */
    RD_ERR_UNSTABLE_DT = 4,       /* dt above the explicit stability bound */
    RD_ERR_WORKSPACE = 5,         /* workspace missing or too small */
    RD_ERR_HIP = 6,               /* a HIP runtime call failed */
    RD_ERR_NONFINITE = 7,         /* a reduction met a NaN or an infinity */
    RD_ERR_NOT_CONVERGED = 8,     /* iteration limit reached before the tolerance */
    RD_ERR_STATE = 9              /* call out of order (e.g. step before bind) */
} rd_status;

typedef enum { RD_FP32 = 0, RD_BF16 = 1, RD_FP16 = 2 } rd_storage;

/* Field layouts (rd_sim_set_layout). */
#define RD_LAYOUT_BLOCKS 0   /* every slot of every stored block (default) */
#define RD_LAYOUT_COMPACT 1  /* only the active voxels of the stored blocks (8^3 blocks) */

/* Workspace features (rd_sim_workspace_bytes). */
#define RD_WS_SOLVER 1u   /* vectors for rd_sim_steady_state */
#define RD_WS_ADJOINT 2u  /* adjoint vectors + checkpoint slots for rd_sim_adjoint */
#define RD_WS_DIFFUSIVITY 4u  /* a per-voxel diffusivity factor (rd_sim_set_diffusivity) */

typedef struct rd_geometry rd_geometry;
typedef struct rd_sim rd_sim;
typedef struct rd_batch rd_batch;

const char *rd_status_string(rd_status s);
const char *rd_last_error(void);

/* ---- geometry (host only; no GPU needed) --------------------------------- */

/* Build the active-block index of a voxel image.
 *   image      host uint8 (nz,ny,nx); nonzero = active voxel (inside Omega, phi > 0)
 *   sdf        host float (nz,ny,nx) signed distance (phi > 0 inside), or NULL.  If
 *              given, (sdf > 0) must equal (image != 0) everywhere, else
 *              RD_ERR_INCONSISTENT_SDF (section "Level-set method", eq. SDF; the
 *              sparse grid holds the points with phi > 0, section "Generating
 *              real-world geometries").
 *   dx         grid spacing (> 0)
 *   block_edge 4 or 8; a block is stored iff it holds an active voxel.
 * Blocks are listed by ascending linear id l = (bz*NBy + by)*NBx + bx,
 * NB = ceil(n / B); slots of a block past the box edge are inactive. */
rd_status rd_geometry_create(const uint8_t *image, const float *sdf, int64_t nx, int64_t ny,
                             int64_t nz, double dx, int block_edge, rd_geometry **out);
/* Counts: active voxels, active blocks, porosity = active / (nx ny nz),
 * fill = active voxels / (active blocks * B^3).  Any output may be NULL. */
rd_status rd_geometry_stats(const rd_geometry *g, int64_t *n_active_vox, int64_t *n_active_blocks,
                            double *porosity, double *fill);
/* Copy the index out: block_id int64[nb] (linear ids, ascending) and nbr
 * int32[nb*6] (list index of the face neighbour in order -x,+x,-y,+y,-z,+z, or -1
 * if outside the box or not stored).  Either may be NULL. */
rd_status rd_geometry_export_index(const rd_geometry *g, int64_t *block_id, int32_t *nbr);
/* Copy the active bitmasks out: uint64[nb * ceil(B^3/64)]; slot (lz*B+ly)*B+lx is
 * bit (slot % 64) of word slot/64 of its block. */
rd_status rd_geometry_export_masks(const rd_geometry *g, uint64_t *masks);
/* Copy the per-slot neighbour codes out: uint8[nb * B^3]; bit d (d = 0..5 in order
 * -x,+x,-y,+y,-z,+z) is set when that face neighbour is an active voxel, bit 6 when
 * the slot itself is active.  The step kernels read these instead of re-deriving
 * neighbour activity from the masks. */
rd_status rd_geometry_export_codes(const rd_geometry *g, uint8_t *codes);
void rd_geometry_destroy(rd_geometry *g);

/* Several geometries stepped together: the time stepping of eq. reaction_diffusion
 * (section "Methods") on many small volumes at once, which then share launches instead
 * of paying a launch each.  rd_geometry_concat builds one geometry whose block list is
 * the parts' lists one after another (neighbour indices shifted, each block tagged with
 * its part); a simulation created on it steps every part in the same kernels, with the same species,
 * reactions, Robin and Dirichlet settings (Dirichlet faces are each part's own box faces),
 * and gives each part the bits it would get alone.  Its dense arrays (rd_sim_set_field,
 * rd_sim_get_field) hold the parts' (nz,ny,nx) boxes one after another, part 0 first.
 * The parts are copied (they may be destroyed afterwards); all need the same block edge
 * and dx; at most 65535 parts.  Calls bound to one box (steady state, adjoint,
 * diffusivity factor, sink band, plane flux, region mass, FRAP) return RD_ERR_STATE on
 * such a simulation.  Errors: RD_ERR_ARG (NULL, n out of range, a part that is itself a
 * concatenation), RD_ERR_SHAPE (mixed block edges or dx, more than 2^31 blocks). */
rd_status rd_geometry_concat(const rd_geometry *const *parts, int n, rd_geometry **out);
/* Number of parts (1 for a geometry built from one image; 0 for NULL). */
int rd_geometry_parts(const rd_geometry *g);
/* Part `part` of a geometry: box shape {nz, ny, nx}, offset of its box in the dense
 * arrays, and its range of blocks in the list.  Outputs may be NULL.  RD_ERR_ARG for a
 * bad part. */
rd_status rd_geometry_part_info(const rd_geometry *g, int part, int64_t shape[3], int64_t *dense_offset,
                                int64_t *first_block, int64_t *n_blocks);

/* ---- signed distance on the GPU --------------------------------------------- */

/* Signed distance of a voxel image (section "Level-set method for image-based geometry
 * reconstruction", eq. SDF; a GPU-built SDF is the future work of section "Discussion
 * and conclusions"), by an exact Euclidean distance transform:
 *   active voxel   (image != 0):  phi = (distance to the nearest inactive voxel centre - 1/2) dx
 *   inactive voxel:               phi = -(distance to the nearest active voxel centre - 1/2) dx
 * and +-(box diagonal) dx when the other phase is empty.  The sign matches the image,
 * so the result passes rd_geometry_create's consistency check, and it feeds
 * rd_sim_set_diffusivity_sdf directly.
 *   dev_image   device uint8 (nz,ny,nx), x fastest
 *   dev_sdf     device float32 (nz,ny,nx), written (caller-owned)
 *   dev_scratch device scratch of rd_sdf_scratch_bytes (20 bytes per voxel, caller-owned)
 * Asynchronous on `stream` (a hipStream_t, NULL = the null stream).  RD_ERR_ARG for
 * NULL pointers or dx <= 0; RD_ERR_SHAPE unless 1 <= n <= 32768 on every axis;
 * RD_ERR_WORKSPACE if the scratch is too small. */
rd_status rd_sdf_scratch_bytes(int64_t nx, int64_t ny, int64_t nz, size_t *bytes);
rd_status rd_sdf_from_image(const uint8_t *dev_image, int64_t nx, int64_t ny, int64_t nz, double dx,
                            float *dev_sdf, void *dev_scratch, size_t scratch_bytes, void *stream);
/* rd_sdf_from_image for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same kernels and the same
 * result, with the scratch taken from a fixed array of 64 MiB that the library holds on
 * each GPU it runs on until the process ends (its device address is fetched once per
 * device, on the first call with that device current).  The caller passes only the
 * image and the output.  No allocation or free happens in the call.  Volumes whose
 * scratch (rd_sdf_scratch_bytes, 20 bytes per voxel, e.g. 144^3) exceeds 64 MiB give
 * RD_ERR_SHAPE; RD_ERR_ARG for NULL pointers or dx <= 0; RD_ERR_HIP if the device or
 * the array's address cannot be obtained.  Every call on one GPU uses that GPU's array,
 * which keeps the previous call's contents (every word is written before it is read):
 * calls that overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  Asynchronous on `stream`. */
rd_status rd_sdf_from_image_static(const uint8_t *dev_image, int64_t nx, int64_t ny, int64_t nz,
                                   double dx, float *dev_sdf, void *stream);

/* ---- simulation ------------------------------------------------------------ */

/* A simulation on geometry g (g must outlive the simulation).  storage selects the
 * field element type in HBM; arithmetic is FP32 and reductions FP64 in every case. */
rd_status rd_sim_create(const rd_geometry *g, rd_storage storage, rd_sim **out);
/* Add a species with diffusion coefficient D >= 0 (at most 4 species); *id receives
 * its index (0, 1, ...).  Must precede rd_sim_bind. */
rd_status rd_sim_add_species(rd_sim *sim, double D, int *id);
/* First-order reaction from -> to at rate >= 0 (to = -1: decay), evaluated at the
 * old time level (law of mass action, section "Methods"). */
rd_status rd_sim_add_reaction(rd_sim *sim, int from, int to, double rate);
/* Wall uptake of a species: flux k * c out through every wall face (k >= 0); the
 * per-face form of the surface-restricted sink of section "Application example 2". */
rd_status rd_sim_set_robin(rd_sim *sim, int species, double k);
/* Hold the active voxels of box face `face` at `value` for a species: the solute
 * that enters the domain from one face (section "Application example 1"; the unit
 * drop between two faces of section "Application example 2").  Those voxels are
 * never updated, act as active neighbours and are left out of the mass.  On edges
 * shared by two flagged faces the higher face id's value wins.  After bind the values
 * are written into the field at once.  RD_ERR_ARG for a bad species or face or a
 * non-finite value. */
rd_status rd_sim_set_dirichlet(rd_sim *sim, int species, int face, double value);
/* Remove every Dirichlet face of a species (same passages; same errors). */
rd_status rd_sim_clear_dirichlet(rd_sim *sim, int species);
/* Launch shape of the time loop (forward Euler steps of section "Discretization and
 * numerical methods"; the paper times one step of its sparse grid, section "Parallel
 * implementation using OpenFPM"): steps per captured graph (>= 1), whether rd_sim_step
 * replays a captured hipGraph (1) or launches directly (0), and whether workgroups
 * are remapped so each of the 8 XCDs walks one contiguous range of the block list
 * (xcd_map = 1; its L2 then holds most halo reads).  Results are bitwise
 * identical for every choice. */
rd_status rd_sim_set_launch(rd_sim *sim, int graph_steps, int use_graph, int xcd_map);
/* Field layout in HBM, before rd_sim_bind (RD_ERR_STATE after it).  The paper stores
 * whole chunks of 8^3 points with an allocation mask (section "Parallel implementation
 * using OpenFPM"); RD_LAYOUT_BLOCKS does the same.  RD_LAYOUT_COMPACT keeps, for every
 * stored block, only its active voxels, block after block in slot order, so a step
 * moves the bytes of the active voxels rather than of whole blocks (the block index,
 * masks and neighbour list are unchanged).  Results are bitwise identical in both
 * layouts.  The compact layout runs the column kernels (2 and 3 of rd_sim_set_kernel)
 * and supports stepping, balances, plane fluxes, region masses and field set/get; a
 * bind with RD_WS_SOLVER, RD_WS_ADJOINT or RD_WS_DIFFUSIVITY returns RD_ERR_STATE.
 * RD_ERR_ARG for an unknown layout; RD_ERR_SHAPE for compact with 4^3 blocks or more
 * than 2^30 - 128 active voxels. */
rd_status rd_sim_set_layout(rd_sim *sim, int layout);
/* Step kernel for B = 8 (ignored for B = 4, which always runs one wave per block):
 *   kernel = 0: one 256-thread workgroup per block;
 *   kernel = 1: persistent, a fixed grid of wg_per_cu * (compute units) workgroups
 *               that walk the block list and prefetch the next block while
 *               computing the current one;
 *   kernel = 2 (default): one wave per block, each lane walking a z-column of 8 voxels;
 *   kernel = 3: as 2, with the x faces of x-adjacent blocks of a workgroup handed
 *               over through LDS instead of being re-read from memory;
 *   kernel = 4: compact layout only: as 2, with buffer accesses (inactive voxels read
 *               as 0 by range checking, no predicates) and the +-x / +-y neighbours
 *               exchanged between lanes (DPP row shifts, ds_bpermute) instead of an
 *               LDS tile.
 * Results are bitwise identical.  RD_ERR_ARG for kernel outside 0..4 or wg_per_cu
 * outside 1..32; RD_ERR_STATE for kernel 0 or 1 with the compact layout and for
 * kernel 4 with the block layout. */
rd_status rd_sim_set_kernel(rd_sim *sim, int kernel, int wg_per_cu);

/* Rounding of the stored fields.  stochastic = 0: round to nearest even (default).
 * stochastic = 1: round up with probability equal to the fraction of the storage
 * spacing, from a counter-based hash of (voxel, species, step, seed): unbiased, so
 * increments below half a spacing are not lost near fronts and steady states.  BF16 /
 * FP16 round so when they store; FP32 storage adds a dither of (u - 1/2) ulp(c) to each
 * voxel's increment before the final addition c + increment is rounded to nearest
 * (constant-D kernels; with a diffusivity factor FP32 stays round-to-nearest).  Results
 * stay deterministic for a given seed and identical across kernels and layouts.
 * Storage precision is an addition of this library; the paper computes in FP32 throughout
 * (section "Parallel implementation using OpenFPM"). */
rd_status rd_sim_set_rounding(rd_sim *sim, int stochastic, uint64_t seed);
/* Device bytes the caller must provide to rd_sim_bind for the given features
 * (bitwise OR of RD_WS_*) and, with RD_WS_ADJOINT, checkpoint_slots stored states.
 * The fields are stored only for the active blocks (section "Parallel implementation
 * using OpenFPM": only chunks holding an inserted point are allocated), two buffers
 * per species.  RD_ERR_ARG for NULL bytes or a negative slot count, RD_ERR_STATE
 * before the first species. */
rd_status rd_sim_workspace_bytes(const rd_sim *sim, uint32_t features, int64_t checkpoint_slots,
                                 size_t *bytes);
/* Attach a caller-owned device workspace (>= the size above, 256-byte aligned) and
 * the stream all work goes to.  Uploads the block index, zeroes the fields and
 * synchronises.  May be called again to move to another workspace (fields reset).
 * The initial condition of every species is 0 with the Dirichlet values applied
 * (section "Application example 1": the solute enters an empty domain).  The caller
 * keeps ownership of the workspace and must keep it alive until the next bind or
 * rd_sim_destroy.  RD_ERR_WORKSPACE if it is NULL, misaligned or too small. */
rd_status rd_sim_bind(rd_sim *sim, void *dev_workspace, size_t bytes, uint32_t features,
                      int64_t checkpoint_slots, void *stream);
/* Scatter a dense device field float32 (nz,ny,nx) into species s; inactive voxels are
 * ignored and Dirichlet voxels take their held value.  This sets the initial condition
 * u(x, 0) of the problem of section "Methods" (eq. reaction_diffusion).  Synchronises;
 * resets the step count.  RD_ERR_ARG for a bad species or NULL pointer, RD_ERR_STATE
 * before bind. */
rd_status rd_sim_set_field(rd_sim *sim, int species, const float *dev_dense);
/* Inhomogeneous diffusion (section "Level-set method for image-based geometry
 * reconstruction", eq. inhomog_diffusion_coefficient; section "Application example
 * 1"; the inhomogeneous-diffusion functor of appendix "Code examples").  A per-voxel
 * factor e makes the diffusion coefficient of species s D_s * e(x); the face between
 * active voxels p and q uses the arithmetic mean D_s (e_p + e_q) / 2, faces toward
 * inactive voxels carry no flux.  dev_dense: device float32 (nz,ny,nx), read at the
 * active voxels only (values there must be finite and >= 0), copied into the
 * workspace (bind with RD_WS_DIFFUSIVITY); the caller keeps ownership.  Synchronises.
 * Afterwards rd_sim_step and rd_sim_balance (Dirichlet inflow with the mean
 * coefficient) use the factor and the stability bound uses D_max * max(e);
 * rd_sim_plane_flux (the mean coefficient on each straddling pair) and rd_sim_adjoint (see
 * rd_sim_adjoint_factor) use it too; rd_sim_steady_state returns RD_ERR_STATE until
 * rd_sim_clear_diffusivity.  Errors: RD_ERR_WORKSPACE without the feature,
 * RD_ERR_STATE before bind, RD_ERR_ARG for a NULL pointer or for invalid values (the
 * factor is then cleared).  A new bind clears the factor. */
rd_status rd_sim_set_diffusivity(rd_sim *sim, const float *dev_dense);
/* As rd_sim_set_diffusivity with e = d_min + d_max / (1 + exp(-(gamma1 + gamma2 phi)))
 * evaluated on the GPU in FP64 (rounded to FP32) from a dense device float32 signed
 * distance phi (nz,ny,nx) (eq. inhomog_diffusion_coefficient; the paper's soil example
 * takes gamma2 = 4h and gamma1 = gamma2 min phi).  RD_ERR_ARG unless d_min, d_max >= 0
 * and all four parameters are finite. */
rd_status rd_sim_set_diffusivity_sdf(rd_sim *sim, const float *dev_sdf, double d_min, double d_max,
                                     double gamma1, double gamma2);
/* Back to the homogeneous D_s. */
rd_status rd_sim_clear_diffusivity(rd_sim *sim);
/* Volumetric sink on a near-surface band (section "Application example 2": a sink
 * restricted to the surface by the level set).  rd_sim_set_sink: rate k_s >= 0 of a
 * species (default 0); on band voxels each step removes dt k_s c (old time level), and
 * rd_sim_balance counts k_s c dx^3 there in the uptake term.  rd_sim_set_sink_band:
 * the band is the set of active voxels with phi < band, phi a dense device float32
 * (nz,ny,nx) (e.g. from rd_sdf_from_image, where the voxels next to the wall have
 * phi = dx/2); *n_band (may be NULL) receives its size; band <= 0 empties it.
 * Needs a bind with RD_WS_DIFFUSIVITY (the band runs through the inhomogeneous
 * kernels, with e = 1 when no factor is set); a new bind empties the band.
 * Synchronises.  The stability bound adds max k_s to the rates; rd_sim_steady_state
 * and rd_sim_adjoint return RD_ERR_STATE while a band with a nonzero rate is set.
 * Errors: RD_ERR_ARG for a bad species, a negative or non-finite rate or band, NULL
 * phi; RD_ERR_WORKSPACE without the feature; RD_ERR_STATE before bind. */
rd_status rd_sim_set_sink(rd_sim *sim, int species, double rate);
rd_status rd_sim_set_sink_band(rd_sim *sim, const float *dev_phi, double band, int64_t *n_band);
/* Simulated FRAP (section "Calculation of effective diffusion coefficient and
 * tortuosity"): the mass of a species inside a box of voxels while the field recovers
 * from a bleached initial state (set with rd_sim_set_field).
 * region = {x0, x1, y0, y1, z0, z1}, half-open voxel index ranges with
 * 0 <= lo < hi <= n on each axis (RD_ERR_ARG otherwise).
 * rd_sim_region_mass: FP64 sum of c dx^3 over the active voxels of the region for the
 * current field (synchronises).  RD_ERR_NONFINITE for a NaN or infinity in the region.
 * rd_sim_frap_curve: curve[k] (host, n_samples + 1 doubles, caller-owned) = the
 * region mass after k * steps_per_sample steps of size dt, k = 0..n_samples (the steps
 * are taken; RD_ERR_UNSTABLE_DT as rd_sim_step). */
rd_status rd_sim_region_mass(rd_sim *sim, int species, const int64_t region[6], double *mass);
rd_status rd_sim_frap_curve(rd_sim *sim, int species, const int64_t region[6], double dt,
                            int64_t steps_per_sample, int64_t n_samples, double *curve);
/* Least-squares effective diffusion coefficient (host only, no GPU): the free-space
 * recovery g was computed with coefficient D_ref at times s_j = j ds (j = 0..m-1); since
 * the diffusion equation depends on D t only, the recovery for coefficient D is
 * g(t D / D_ref), linearly interpolated.  D_eff minimises
 * sum_i (f_i - g(t_i D / D_ref))^2 over D in [1e-4, 1] * D_ref (m-1) ds / max t (a
 * 400-point log scan, then golden-section search); rms = sqrt(minimum / n), may be NULL.
 * Inputs are host arrays: t, f of n samples (t >= 0, one t > 0), g of m.  The
 * tortuosity of eq. tortuosity is tau_d = D / D_eff.  RD_ERR_ARG for n or m < 2, ds or
 * D_ref <= 0, non-finite values. */
rd_status rd_frap_fit(int64_t n, const double *t, const double *f, int64_t m, double ds,
                      const double *g, double D_ref, double *D_eff, double *rms);
/* Gather species s into a dense device float32 (nz,ny,nx) (a concatenated geometry: the
 * parts' boxes one after another); inactive voxels -> 0. */
rd_status rd_sim_get_field(const rd_sim *sim, int species, float *dev_dense);
/* Advance n_steps FTCS steps of size dt (asynchronous).  RD_ERR_UNSTABLE_DT if
 * dt > 2 / lambda_max with the Gershgorin bound
 * lambda_max = 12 D_max/dx^2 + max_a(total rate out of a) + 6 max_a(k_R,a)/dx
 * (the 3-D form of the paper's eq. diffusion_stability_condition). */
rd_status rd_sim_step(rd_sim *sim, double dt, int64_t n_steps);
/* Steps taken since bind / the last set_field. */
rd_status rd_sim_steps_taken(const rd_sim *sim, int64_t *n);
/* FP64 balance terms of species s for the current field (synchronises):
 *   mass   = sum over free voxels of c dx^3
 *   inflow = sum over Dirichlet voxels q and free active neighbours p of D (c_q - c_p) dx
 *   uptake = sum over free voxels of k_R n_wall c dx^2
 * With them one step satisfies M' - M = dt (inflow - uptake + reactions).
 * RD_ERR_NONFINITE if the field holds a NaN or infinity.  Outputs may be NULL. */
rd_status rd_sim_reduce(rd_sim *sim, int species, double *mass, double *dirichlet_inflow,
                        double *robin_uptake);
/* All balance terms: out[0] mass, out[1..6] inflow per face, out[7] uptake,
 * out[8] reaction total (sum over free voxels of the reaction rate, times dx^3). */
rd_status rd_sim_balance(rd_sim *sim, int species, double out[9]);
/* rd_sim_balance over the blocks of one part of a concatenated geometry
 * (rd_geometry_concat); part 0 of a single geometry is the whole.  RD_ERR_ARG for a bad
 * part. */
rd_status rd_sim_balance_part(rd_sim *sim, int species, int part, double out[9]);
/* Diffusive flux of a species through the plane between indices i0 and i0 + 1 along
 * `axis` (0 x, 1 y, 2 z), positive in the +axis direction (the flux from which an
 * effective diffusivity, and with it the tortuosity of eq. background:tortuosity, is
 * read):  sum over pairs (p, p + e_axis) of active voxels of D (c_p - c_{p+e}) dx,
 * accumulated in FP64 in a fixed order (synchronises).  RD_ERR_ARG unless
 * 0 <= i0 < n_axis - 1; RD_ERR_STATE before bind. */
rd_status rd_sim_plane_flux(rd_sim *sim, int species, int axis, int64_t i0, double *flux);

/* Steady state of species 0 (single-species, no reactions or Robin) with a unit
 * drop along `axis` (Dirichlet 1 on the low face plane, 0 on the high one,
 * no-flux elsewhere), solved by conjugate gradients with the stencil as operator
 * (the FTCS step's operator at t -> infinity), a block-Jacobi preconditioner
 * (rd_sim_set_cg_precond) and FP64 dot products.  Initial guess:
 * the linear ramp on 6-connected clusters touching both planes, 1 on clusters touching
 * only the inlet, 0 on the rest (clusters labelled on the GPU).  The iterate is kept in
 * FP64; every 25 iterations the FP64 residual b - A x is evaluated (rel_residual is its
 * norm over ||b||) and replaces the recursive residual when the two have drifted apart
 * (with 16-bit vectors a replacement also restarts the search direction), so 1e-8 is
 * reachable with FP32, BF16 or FP16 vectors.  Stops at rel. residual <=
 * rel_tol (RD_OK), or at stagnation (no 10% decrease of the best residual over 40
 * checks, i.e. 1000 iterations: CG's residual is not monotone and plateaus for
 * hundreds of iterations on large volumes) or max_iters (RD_ERR_NOT_CONVERGED, outputs
 * still written).
 * tau = psi D A / (Q L): psi active fraction, A box cross-section, L = (n-1) dx,
 * Q the mean of the inflow at the inlet plane and the outflow at the outlet plane of
 * the FP64 iterate (equal at an exact steady state; eq. tortuosity, tau = D_f / D_eff);
 * +inf if no cluster touches both planes or Q <= 0.  Needs RD_WS_SOLVER.  Leaves the
 * steady field (the FP64 iterate rounded to the storage type) in species 0. */
rd_status rd_sim_steady_state(rd_sim *sim, int axis, double rel_tol, int64_t max_iters,
                              double *tau, double *rel_residual, int64_t *iters);

/* Preconditioner of the steady-state CG (eq. tortuosity needs only the converged field,
 * so the preconditioner changes the path to it, not the result).  With 8^3 blocks,
 * jacobi_steps >= 1 runs preconditioned CG with M^-1 r = jacobi_steps Jacobi steps on
 * each block's own equations (the diagonal of the operator, the block's own free
 * neighbours; neighbours outside the block count as 0): a symmetric positive definite
 * polynomial in the block operator, applied in the registers of the update kernel (one
 * more vector written per iteration).  Even counts condition best; 0 = plain CG.
 * Default 6; 4^3 blocks always run plain CG.  RD_ERR_ARG for NULL or a count outside
 * 0..16.  rd_batch_set_cg_precond sets the same for a batch. */
rd_status rd_sim_set_cg_precond(rd_sim *sim, int jacobi_steps);

/* Discrete adjoint of a single-species diffusion-decay simulation (optionally with
 * Robin walls and Dirichlet faces), run from the current field for n_steps of size
 * dt.  Gradients with respect to D and to the decay rate k (the sum of the rates of
 * its decay reactions; 0 if none):
 *   seed_mode 0: dev_seed is a target c* (dense float32 (nz,ny,nx));
 *                L = 1/2 sum over free voxels of (c^N - c*)^2, returned in *loss;
 *   seed_mode 1: dev_seed is dL/dc^N (dense float32); *loss = 0.
 * The recursion lambda^n = J^T lambda^{n+1} uses the symmetry of the step's
 * Jacobian J (mirror rule); dL/dD = sum_n dt/dx^2 <lambda^{n+1}, L c^n>,
 * dL/dk = -sum_n dt <lambda^{n+1}, c^n>, accumulated in FP64.  States are
 * checkpointed every `checkpoint_every` = k steps and recomputed per segment:
 * needs RD_WS_ADJOINT with checkpoint_slots >= ceil(n_steps / k) + k - 1, and
 * round-to-nearest storage.  With a diffusivity factor set, L is the factor-weighted
 * Laplacian (face coefficient (e_p + e_q) / 2) in both the recursion and dL/dD; an
 * active sink band (nonzero rate) gives RD_ERR_STATE.  On return species 0 holds c^N. */
rd_status rd_sim_adjoint(rd_sim *sim, const float *dev_seed, int seed_mode, int64_t n_steps,
                         double dt, int checkpoint_every, double *loss, double *dL_dD,
                         double *dL_drate);
/* rd_sim_adjoint with a diffusivity factor set (rd_sim_set_diffusivity), adding the
 * gradient of the loss with respect to the factor of every voxel:
 *   dev_dL_de  device double (nz,ny,nx), caller-owned, written (0 off the active voxels):
 *              dL/de_p = sum_n (D dt / dx^2) / 2 * sum_{q active nb of p}
 *                        (c^n_q - c^n_p)(lambda^{n+1}_p - lambda^{n+1}_q),
 * lambda being 0 on Dirichlet voxels.  The factor's parameters follow by the chain rule;
 * for e = D_min + D_max s(g1 + g2 phi), s the logistic function,
 * dL/dg1 = sum_p dL/de_p D_max s (1 - s) and dL/dg2 = sum_p dL/de_p D_max s (1 - s) phi_p
 * (eq. inhomog_diffusion_coefficient).  dL/dD, dL/drate and the loss as rd_sim_adjoint,
 * whose recursion with a factor uses the face coefficient (e_p + e_q) / 2.  Needs a bind
 * with RD_WS_ADJOINT | RD_WS_DIFFUSIVITY (RD_ERR_WORKSPACE), a factor (RD_ERR_STATE),
 * no active sink band (RD_ERR_STATE); RD_ERR_ARG for NULL dev_dL_de; otherwise the
 * errors of rd_sim_adjoint. */
rd_status rd_sim_adjoint_factor(rd_sim *sim, const float *dev_seed, int seed_mode, int64_t n_steps,
                                double dt, int checkpoint_every, double *loss, double *dL_dD,
                                double *dL_drate, double *dev_dL_de);
/* Change a species' D, or the rate of reaction `index` (in order of addition), after
 * binding (used between differentiable runs). */
rd_status rd_sim_set_species_D(rd_sim *sim, int species, double D);
rd_status rd_sim_set_reaction_rate(rd_sim *sim, int index, double rate);
void rd_sim_destroy(rd_sim *sim);

/* ---- autotuning ----------------------------------------------------------- */

/* Time every launch configuration of a bound simulation (steps per captured graph
 * 16 or 64; plain or XCD-aware block order; for B = 8 the workgroup-per-block and
 * z-column kernels, and the persistent kernel with 2, 4 or 8 workgroups per CU) on
 * `trial_steps` steps of size dt, with HIP events on
 * the bound stream, and keep the fastest.  All configurations give bitwise-identical
 * fields.  The trials advance the fields, so the simulation is reset afterwards
 * (fields zero, Dirichlet values applied): call it before rd_sim_set_field.
 * *best_ms (may be NULL) receives the mean time per step of the chosen setting. */
rd_status rd_sim_autotune(rd_sim *sim, double dt, int64_t trial_steps, double *best_ms);
/* rd_sim_autotune with a result cache, for callers that bind the same geometry again
 * and should not pay the trials every time.  The key
 * covers the GPU (architecture and compute units), storage type, species count,
 * reactions, Robin walls and the geometry (extents, block edge, every activity word).
 * A cache hit applies the stored launch configuration without trials and leaves the
 * fields untouched; a miss runs rd_sim_autotune (which resets the fields) and appends
 * one text line "rdtune1 <key> <kernel> <xcd> <graph> <wg_per_cu> <graph_steps> <ms>" to
 * cache_path (created if missing; the last line of a key wins).  *from_cache and
 * *best_ms may be NULL.  RD_ERR_ARG if the file cannot be written. */
rd_status rd_sim_autotune_cached(rd_sim *sim, double dt, int64_t trial_steps, const char *cache_path,
                                 int *from_cache, double *best_ms);
/* Autotune each candidate simulation (for example the same image indexed with 4^3 and
 * with 8^3 blocks, same species and parameters) and report the fastest:
 * *best_index, and ms_per_step[n] (may be NULL). */
rd_status rd_autotune_pick(rd_sim *const *sims, int n, double dt, int64_t trial_steps,
                           int *best_index, double *ms_per_step);
/* Steps per launch (1..256, default 1): with more than one, rd_sim_step issues the steps
 * in cooperative launches of that many steps each, a grid barrier between the steps
 * (the explicit steps of eq. reaction_diffusion, section "Methods", unchanged and in
 * order; what goes is the launch per step, which dominates small volumes).  The fields
 * are those of one launch per step bit for bit.  Applies to 8^3
 * blocks in the block layout with a column kernel (rd_sim_set_kernel 2 or 3) and constant
 * D; other settings keep one launch per step.  Fused launches are not captured in graphs.
 * RD_ERR_ARG outside 1..256, RD_ERR_STATE for 4^3 blocks or the compact layout. */
rd_status rd_sim_set_fused_steps(rd_sim *sim, int steps);
rd_status rd_sim_get_fused_steps(const rd_sim *sim, int *steps);
/* Current launch configuration (any output may be NULL). */
rd_status rd_sim_get_launch(const rd_sim *sim, int *graph_steps, int *use_graph, int *xcd_map,
                            int *kernel, int *wg_per_cu);

/* ---- batches of geometries ------------------------------------------------- */

/* Many geometries solved together: the tortuosity of eq. tortuosity (section
 * "Calculation of effective diffusion coefficient and tortuosity") of each geometry,
 * from the steady unit-drop problem of rd_sim_steady_state.  Their block lists are
 * concatenated and one launch per kernel stage covers every geometry.  Single
 * species, D = 1, pure diffusion.  The geometries must outlive the batch.  RD_ERR_ARG
 * unless 1 <= n <= 65535, for a NULL geometry or an unknown storage type;
 * RD_ERR_SHAPE if the block edges differ or the batch holds 2^31 blocks or more. */
rd_status rd_batch_create(const rd_geometry *const *geoms, int n, rd_storage storage,
                          rd_batch **out);
/* Device bytes of a batch's workspace (same storage rule as rd_sim_workspace_bytes:
 * active blocks only, plus the solver vectors), and its binding (caller-owned
 * workspace, 256-byte aligned, kept alive by the caller; the stream as in rd_sim_bind;
 * RD_ERR_WORKSPACE if NULL, misaligned or too small). */
rd_status rd_batch_workspace_bytes(const rd_batch *b, size_t *bytes);
rd_status rd_batch_bind(rd_batch *b, void *dev_workspace, size_t bytes, void *stream);
/* Per-geometry tortuosity along `axis` by batched conjugate gradients (one launch
 * per kernel stage for the whole batch), with the initial guess, FP64 iterate,
 * residual replacement and stopping rule of rd_sim_steady_state applied per geometry;
 * converged geometries stop updating.  tau[n], rel_residual[n], iters[n] are host
 * arrays (any may be NULL).  RD_ERR_NOT_CONVERGED if any geometry stopped above
 * rel_tol (outputs still written). */
rd_status rd_batch_tortuosity(rd_batch *b, int axis, double rel_tol, int64_t max_iters,
                              double *tau, double *rel_residual, int64_t *iters);
/* Launch setting of a batch's CG: iters_per_check (1..1000, default 25) iterations run
 * between two FP64 residual checks (the convergence test, which reads scalars back to the
 * host) as one sequence of launches, replayed as a captured hipGraph when use_graph is 1
 * (default) or launched directly.  The stagnation rule counts 1000 iterations whatever
 * the interval.  RD_ERR_ARG for a NULL batch or an interval outside 1..1000. */
rd_status rd_batch_set_launch(rd_batch *b, int iters_per_check, int use_graph);
rd_status rd_batch_get_launch(const rd_batch *b, int *iters_per_check, int *use_graph);
/* The preconditioner of a batch's CG, as rd_sim_set_cg_precond (default 6). */
rd_status rd_batch_set_cg_precond(rd_batch *b, int jacobi_steps);
/* Autotuning of batches: bound candidate batches of the same geometries (indexed with
 * different block edges, say) each try iters_per_check 25 and 50 with and without graph
 * replay, running max(trial_iters, interval) CG iterations along `axis` per trial, and
 * keep their fastest setting; the wall time per iteration, net of labelling and initial
 * guess, of each candidate's best setting goes to ms_per_iter[n] (may be NULL) and the
 * fastest candidate's index to *best_index.  The workspaces' contents are overwritten. */
rd_status rd_batch_autotune_pick(rd_batch *const *batches, int n, int axis, int64_t trial_iters,
                                 int *best_index, double *ms_per_iter);
void rd_batch_destroy(rd_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* RD_H */
