/*
 * sbpfdtd: the leapfrog E/H step of the 3D SBP-SAT FDTD method
 * (Cheng, Liu et al., "Towards the Development of a Three-Dimensional
 * SBP-SAT FDTD Method: Theory and Validation"), native HIP for gfx950.
 *
 * C ABI.  Plain pointers and sizes; no C++ or torch types.  Every call
 * returns an sbp_status; no exception or abort crosses the ABI.  The last
 * error message of a context is available from sbp_last_error().
 *
 * Conventions
 *  - Cells of a block are indexed (i, j, k), i fastest.  Field components
 *    live on the grids of Table T1: Ex on (x-, y+, z+), Ey (x+, y-, z+),
 *    Ez (x+, y+, z-), Hx (x+, y-, z-), Hy (x-, y+, z-), Hz (x-, y-, z+); a
 *    "+" axis of n cells has n+1 nodes (x_i = i h), a "-" axis n+2 nodes
 *    (0, h/2, 3h/2, ..., nh) (Section II-A).  Node arrays are i fastest.
 *  - Faces: 0 = -x, 1 = +x, 2 = -y, 3 = +y, 4 = -z, 5 = +z.
 *  - Host arrays passed in are copied during the call; the caller keeps
 *    ownership.  Device memory is taken from the allocator callbacks given
 *    to sbp_create (or hipMalloc when they are NULL) and returned on
 *    sbp_destroy.
 *  - sbp_step() only enqueues work on the context's stream; the read calls
 *    synchronise that stream and copy into caller memory (fp32 fields are
 *    widened to double).
 *  - A context is used from one host thread at a time.
 */
#ifndef SBPFDTD_H
#define SBPFDTD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbp_ctx sbp_ctx;

typedef enum {
  SBP_OK = 0,
  SBP_EINVAL = -1,     /* bad argument (sizes, indices, face pairing, ratio) */
  SBP_ENOMEM = -2,     /* device allocation failed */
  SBP_EHIP = -3,       /* a HIP runtime call failed */
  SBP_ESTATE = -4,     /* call out of order (e.g. step before finalize) */
  SBP_EUNSTABLE = -5,  /* time step above the stability limit, or non-finite energy */
  SBP_ERANGE = -6      /* requested samples not (or no longer) available */
} sbp_status;

typedef enum { SBP_FP64 = 0, SBP_FP32 = 1 } sbp_prec;

/* Face treatments (Section III): PEC and PMC penalties (E13-E15 / E18,
 * E19-E21 / E23); SBP_ABC1 is a first-order absorbing (characteristic)
 * penalty, which the paper does not have; SBP_CPML is a PEC face behind a
 * convolutional perfectly matched layer (the truncation of the paper's
 * Section VI examples; see sbp_set_cpml). */
typedef enum { SBP_PEC = 0, SBP_PMC = 1, SBP_ABC1 = 2, SBP_CPML = 3 } sbp_bc;

typedef enum { SBP_EX = 0, SBP_EY, SBP_EZ, SBP_HX, SBP_HY, SBP_HZ } sbp_comp;

/* Source waveforms of Section VI: 0 = Gaussian pulse exp(-4 pi (t-t0)^2/tw^2),
 * 1 = the same times sin(2 pi f0 t). */
typedef enum { SBP_GAUSS = 0, SBP_MODGAUSS = 1 } sbp_wave;

typedef void *(*sbp_alloc_fn)(size_t bytes, void *user);
typedef void (*sbp_free_fn)(void *ptr, void *user);

/* Creates a context: the leapfrog state of Section V (E^n and H^{n-1/2} on
 * the grids of Table T1, for every block added) computed in `prec` on HIP
 * stream `hip_stream` (NULL = default stream) of the current device.
 * `alloc`/`free_fn` may be NULL (hipMalloc/hipFree). */
sbp_status sbp_create(sbp_ctx **out, sbp_prec prec, void *hip_stream,
                      sbp_alloc_fn alloc, sbp_free_fn free_fn, void *user);

/* Adds a block of nx*ny*nz cells (each >= 4: the boundary closures of the
 * Appendix need four cells; one component array, the node box
 * (nx+2)(ny+2)(nz+2) with its xy planes padded to 64 nodes, must stay below
 * 4 GiB: about 1000^3 cells in fp32, 800^3 in fp64) of size dx*dy*dz metres
 * at origin (x0,y0,z0).
 * eps_r, mu_r, sigma (S/m): per-cell host arrays of nx*ny*nz doubles, i
 * fastest, or NULL for 1, 1, 0.  The node value is the mean over the cells
 * whose closed box contains the node.  All faces start as PEC. */
sbp_status sbp_add_block(sbp_ctx *ctx, int nx, int ny, int nz, double dx, double dy,
                         double dz, double x0, double y0, double z0, const double *eps_r,
                         const double *mu_r, const double *sigma, int *block_id);

/* Sets the treatment of one outer face of a block. */
sbp_status sbp_set_face_bc(sbp_ctx *ctx, int block, int face, sbp_bc bc);

/* Couples face_a of blk_a with face_b of blk_b (opposite faces of one axis,
 * covering each other exactly) through interface penalties: the pattern of
 * EPBC1-EPBC6 with zero phase and sigma = chi = +-1/2 (EPBCP).  ratio = cells
 * of blk_b per cell of blk_a along the face, 1 or 2; at 2 the neighbour's
 * face values are interpolated by a norm-compatible pair of operators. */
sbp_status sbp_connect(sbp_ctx *ctx, int blk_a, int face_a, int blk_b, int face_b, int ratio);

/* Makes both faces of `axis` (0 = x, 1 = y, 2 = z) of `block` periodic
 * (Section III, EPBC1-EPBC6 with sigma = chi = +-1/2 of EPBCP): each face is
 * penalised with the opposite face's values, the high face with e^{-j alpha}
 * times the low face's and the low face with e^{+j alpha} times the high
 * face's, alpha = k0_axis times the block length along the axis.
 *   block_im < 0: real fields; alpha must be 0.
 *   block_im >= 0: the fields are complex, `block` holding the real and
 *     `block_im` the imaginary part.  The two blocks must have the same cells
 *     and spacings (and should be given the same materials); the call makes
 *     the axis periodic in both, with the parts mixed by cos / sin alpha at
 *     the faces.  Every periodic axis of a complex block names the same
 *     block_im (alpha may be 0 on some axes), and the two parts take no
 *     interfaces (sbp_connect).  W^n is then the energy of the complex field.
 * Errors: SBP_EINVAL for a bad block or axis, a non-finite alpha, alpha != 0
 * without block_im, mismatched parts, a block paired with two different
 * partners (or as both the real and the imaginary part), a complex block
 * with interfaces, or a face already coupled; SBP_ESTATE after
 * sbp_finalize. */
sbp_status sbp_set_periodic(sbp_ctx *ctx, int block, int block_im, int axis, double alpha);

/* Total-field / scattered-field plane-wave injection (Section VI brings
 * the incident wave of its examples in this way).  `box` = {ilo, ihi, jlo,
 * jhi, klo, khi} is a box of cells of `block`, at least 4 cells inside it on
 * every side (and at least cells + 4 inside any SBP_CPML face); nodes on or
 * inside it carry the total field, the others the scattered field.  Each
 * difference that couples nodes of the two regions takes the neighbour's
 * value in the node's own convention, i.e. adds or removes the incident
 * field there (inside the Cb bracket for E).  The incident wave travels
 * along +axis with E along `pol` (an E component across the axis); it comes
 * from a one-dimensional line stepped on the device with the same dt, h,
 * eps0 and mu0 (the interior difference of the axis; PEC ends) over node
 * indices -margin .. n[axis] + margin, driven by a soft current source of
 * waveform `w`, p = {tw, t0, f0}, on line node src_cell (in
 * 1 - margin .. n[axis] + margin - 1), evaluated at (n+1/2) dt.  The line is
 * part of the saved state.  One box per context, before sbp_finalize; the
 * block takes no interface or periodic faces; sbp_adjoint rejects it.
 * Errors: SBP_EINVAL for a bad block, axis, polarisation, box, margin
 * (1 .. 2^20), source cell, waveform or width (and at sbp_finalize for a box
 * too close to absorbing layers or a block with interface or periodic
 * faces); SBP_ESTATE for a second box or after sbp_finalize. */
sbp_status sbp_set_tfsf(sbp_ctx *ctx, int block, const int box[6], int axis, sbp_comp pol, int margin,
                        int src_cell, sbp_wave w, const double p[3], double amplitude);

/* Layer parameters of the faces set to SBP_CPML (before sbp_finalize; the
 * defaults are 10, 3, 0.8, 1, 0).  Inside a layer of `cells` cells next to
 * such a face every difference along the face normal (the SBP operator with
 * its closure rows and the face's PEC penalty) becomes d/kappa + psi, with
 * psi <- b psi + c d advanced once per half step.  At depth rho in [0, 1]
 * into the layer (1 on the face): sigma = sigma_factor (order+1)/(eta0 h)
 * rho^order, kappa = 1 + (kappa_max - 1) rho^order, alpha = alpha_max
 * (1 - rho) (S/m); b = exp(-(sigma/kappa + alpha) dt/eps0), c = sigma (b - 1)
 * / (sigma kappa + kappa^2 alpha), at each node's own position (grids of
 * Table T1).  The psi are part of the saved state.  Blocks with layers are
 * rejected by sbp_adjoint.  Errors: SBP_EINVAL for cells < 1, order outside
 * 1..8, sigma_factor < 0, kappa_max < 1 or alpha_max < 0; SBP_ESTATE after
 * sbp_finalize. */
sbp_status sbp_set_cpml(sbp_ctx *ctx, int cells, int order, double sigma_factor, double kappa_max,
                        double alpha_max);

/* Soft source (a current density inside the E update) on node (i,j,k) of an
 * E component; p = {tw, t0, f0} in seconds / Hz; evaluated at (n+1/2) dt. */
sbp_status sbp_add_source(sbp_ctx *ctx, int block, sbp_comp c, int i, int j, int k,
                          sbp_wave waveform, const double p[3], double amplitude, int *id);

/* Probe of one node per step (the field records of Section VI's examples):
 * sample n is E^{n+1} (or H^{n+1/2}), node (i,j,k) on the component's grid
 * of Table T1. */
sbp_status sbp_add_probe(sbp_ctx *ctx, int block, sbp_comp c, int i, int j, int k, int *id);

/* Builds the plan and device buffers.  dt = cfl_fraction times the Yee limit
 * of the finest block (the limit the paper reports for its SBP-SAT scheme,
 * Section VI-A).  cfl_fraction > 1 gives SBP_EUNSTABLE unless `force` != 0.
 * history = number of per-step energy / probe samples retained (ring). */
sbp_status sbp_finalize(sbp_ctx *ctx, double cfl_fraction, int force, long history,
                        double *dt_out);

/* Replaces the per-cell materials of a block after finalize (NULL = 1,1,0):
 * the eps, mu and sigma of E7-E12 and Section V's lossy update, formed per
 * node as the mean of the cells containing the node, as at sbp_add_block. */
sbp_status sbp_set_materials(sbp_ctx *ctx, int block, const double *eps_r, const double *mu_r,
                             const double *sigma);

/* Enqueues nsteps leapfrog steps (H half step, then E step, Section V). */
sbp_status sbp_step(sbp_ctx *ctx, long nsteps);

/* Allocation-free stepping, for callers that cannot allocate device memory
 * while they step (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The same steps as sbp_step (bitwise
 * equal fields, probes and energies), but the per-step scratch of the
 * kernels (the energy partial sums of every launch and the interface face
 * buffers) lives in a fixed device array of 16 MiB per GPU (2 MiB of partial
 * sums, 14 MiB of face values), set up by sbp_create, instead of buffers of
 * the context.  Eager launches only: no graph is captured or replayed and no
 * timing events are recorded (sbp_last_step_ms does not cover these steps).
 * Calls no allocating routine.  Returns SBP_EINVAL, before enqueuing
 * anything, if the context's launch shape needs more than 262144 partial
 * sums or its interfaces more than 1835008 face values (then use sbp_step).
 * Every context on a GPU uses that GPU's one array, which keeps the last
 * call's contents; each call first clears the face-buffer part (with a
 * kernel, no memset), and every partial sum is written before it is read.
 * Calls that overlap in time on one GPU, from different streams or threads,
 * race and must be serialised by the caller. */
sbp_status sbp_step_static(sbp_ctx *ctx, long nsteps);

/* Number of steps taken so far. */
sbp_status sbp_steps_done(const sbp_ctx *ctx, long *n);

/* Local time stepping at 1:p for refined blocks.  The paper leaves the
 * coupling of blocks of different mesh sizes to later work (Sections I and
 * VII); the scheme here is the explicit, energy-conserving two-level local
 * time stepping of Diaz and Grote on the E-only form of Section V's lossless
 * leapfrog, E^{n+1} - 2 E^n + E^{n-1} = -dt^2 L E^n, L = -eps^-1 K_eh mu^-1
 * K_he (E7-E12 with the SAT rows).  With P the projector onto the E nodes of
 * the blocks listed in `refined`, a coarse step of length dt_coarse takes
 * w = L (I - P) E^n and `substeps` substeps of dt_coarse / substeps in which
 * only P q changes, then E^{n+1} = -E^{n-1} + 2 q_p, so the refined blocks
 * advance with the short step and the others with the coarse one.  The
 * scheme conserves W^{n+1/2} = 1/2 |E^{n+1} - E^n|_M^2 / dt^2
 * + 1/2 <E^{n+1}, M (2 E^n - E^{n+1} - E^{n-1})> / dt^2 (M the E16 weights
 * times eps); substeps = 1, or no refined block, is the leapfrog.
 * It runs as the ordinary step of length dt_coarse on every block plus a
 * correction on the refined blocks and the nodes of other blocks within a
 * few cells of them; the H arrays hold the auxiliary H^{n+1/2} = H^{n-1/2}
 * + dt B E^n of that step, which equals the leapfrog's H only where no
 * correction has reached.
 * sbp_lts_start takes the current state (E^0, H^{-1/2}); sbp_lts_step
 * enqueues nsteps coarse steps, advancing the step index by one per coarse
 * step.  With energy_every = K > 0, energy slot n holds W^{n+1/2} for the
 * steps n that K divides and NaN for the others (K = 0: NaN throughout);
 * forming it reads every E array twice more.  The context then holds E^n
 * (read with sbp_read_field) and steps only by sbp_lts_step: sbp_step,
 * sbp_step_static, sbp_save_state, sbp_load_state, sbp_write_field,
 * sbp_set_materials, sbp_set_fused, sbp_set_cell_tables, sbp_autotune and
 * sbp_adjoint return SBP_ESTATE.  Device memory for up to seven more field
 * pools is taken at sbp_lts_start.  Errors: SBP_EINVAL for
 * substeps outside 1..64, a non-positive dt_coarse, a negative energy_every,
 * a bad refined block, a lossy block (conductivity, absorbing face or
 * layer), periodic faces, sources, probes, a TF/SF box or the one-pass step;
 * SBP_ESTATE before sbp_finalize or on a second sbp_lts_start. */
sbp_status sbp_lts_start(sbp_ctx *ctx, const int *refined, int nrefined, int substeps, double dt_coarse,
                         long energy_every);
sbp_status sbp_lts_step(sbp_ctx *ctx, long nsteps);
/* The extent of the correction of local time stepping: out[0] tiles of the
 * correction's operator steps of all out[1] tiles of a step, out[2] nodes in
 * the near boxes (the refined blocks whole, and the nodes of other blocks
 * within three of their cells of a refined block) of all out[3] nodes of the
 * node boxes.  SBP_ESTATE before sbp_lts_start. */
sbp_status sbp_lts_info(const sbp_ctx *ctx, long out[4]);

/* Node counts (Sx, Sy, Sz) of a component of a block. */
sbp_status sbp_field_shape(const sbp_ctx *ctx, int block, sbp_comp c, int shape[3]);

/* Copies a component to / from host doubles (Sx*Sy*Sz on the component's
 * grid of Table T1, i fastest).  Writing sets E^n or H^{n-1/2} of the
 * current step (the leapfrog state of Section V). */
sbp_status sbp_read_field(sbp_ctx *ctx, int block, sbp_comp c, double *dst, size_t count);
sbp_status sbp_write_field(sbp_ctx *ctx, int block, sbp_comp c, const double *src, size_t count);

/* Energy W^n (E16, leapfrog pairing of H) for n = first .. first+count-1. */
sbp_status sbp_read_energy(sbp_ctx *ctx, long first, long count, double *dst);

/* Probe samples n = first .. first+count-1 of probe `id`. */
sbp_status sbp_read_probe(sbp_ctx *ctx, int id, long first, long count, double *dst);

/* Device-to-device snapshot of the time-stepping state (Section V's E^n
 * and H^{n-1/2}, with the step index n), the CPML recursion variables and the
 * TF/SF incident line.
 * bytes must be >= sbp_state_bytes(); sbp_load_state restores a snapshot of
 * the same context (the sources' values follow from the step index). */
sbp_status sbp_state_bytes(const sbp_ctx *ctx, size_t *bytes);
sbp_status sbp_save_state(sbp_ctx *ctx, void *dev_buf, size_t bytes);
sbp_status sbp_load_state(sbp_ctx *ctx, const void *dev_buf, size_t bytes);

/* Gradient of a region objective with respect to the per-cell relative
 * permittivity, by the discrete adjoint of the leapfrog step (Section V):
 *   J = dt * sum_{n=1..N} sum_{cells c in region} |Ebar_c^n|^2,
 * with E^n the fields n steps after the current state and Ebar_c, per
 * component, the mean of the four edges of cell c that carry it.  The
 * forward run (N = nsteps steps) stores its state every ckpt_every steps
 * (0 = ceil(sqrt(N))); the reverse sweep recomputes each segment from its
 * checkpoint and runs the adjoint backwards through it.  region = {i0, i1,
 * j0, j1, k0, k1}: half-open cell box of `block`.  Writes J to *J_out (host)
 * and dJ/d eps_r of every cell of `block` to grad_eps_dev (device doubles,
 * nx*ny*nz, i fastest; the caller owns it); the cell sums run in a fixed
 * order, so repeated calls give the same bits.  grad_eps_dev = NULL
 * evaluates J alone (the forward run; no checkpoints, no reverse sweep, one
 * double of device memory).  Blocks must be lossless (no
 * conductivity, no absorbing faces): SBP_EINVAL otherwise.  Afterwards the
 * context is at the state after the N forward steps, with their energy and
 * probe samples, as after sbp_step(ctx, N).  Device memory for
 * ceil(N/ckpt_every) states plus ckpt_every+1 field pools is taken from the
 * allocator and returned before the call ends; SBP_ENOMEM if it is not
 * available. */
sbp_status sbp_adjoint(sbp_ctx *ctx, int block, long nsteps, const int region[6], long ckpt_every,
                       double *J_out, double *grad_eps_dev);

/* Launch shape of the step kernels: a tile is cz runs of tx*ty consecutive
 * nodes of a block's node box in flat order (i fastest, then j, then k), one
 * node per thread and run; `workgroups` resident workgroups loop over the
 * tile list (0 = one workgroup per tile).  tx*ty must be 64, 128 or 256;
 * 1 <= cz <= 1024.  Without this call (or sbp_autotune) the shape is
 * 128, 1, 8, 0, with fewer planes per tile when the blocks give few tiles of
 * 8 planes: 4 below 2048 such tiles, 2 below 512 and 1 below 160. */
sbp_status sbp_set_launch(sbp_ctx *ctx, int tx, int ty, int cz, int workgroups);
sbp_status sbp_get_launch(const sbp_ctx *ctx, int out[4]);

/* Storage of the per-cell permittivity that the E update reads (E7-E9: Cb
 * from the sum of the four cells around an E node).  A plain block (PEC /
 * PMC faces, no conductivity, no per-cell permeability, no interfaces, no
 * TF/SF box) whose cells take at most 64 distinct values in the field
 * precision also holds them as one byte per cell, an index into a table of
 * those values, and its E update reads the bytes (1 B per cell instead of 4
 * (fp32) or 8 (fp64)) when the launch shape takes one workgroup per tile of
 * 8 or more planes.  The values, and so every result, are the same either
 * way.  enable != 0 (the default) tables the blocks that qualify, enable = 0
 * keeps every block on the cell array.  Before or after sbp_finalize
 * (afterwards the tile lists are rebuilt and a captured step graph is
 * dropped); SBP_ESTATE under local time stepping. */
sbp_status sbp_set_cell_tables(sbp_ctx *ctx, int enable);

/* Selects how plain blocks (PEC / PMC faces, no conductivity, no per-cell
 * permeability, no interfaces) are stepped: enable != 0 runs both half steps
 * in one pass over the fields (each value read and written once per step),
 * on windows of 32 x 8 node columns walking `planes` planes (4..4096);
 * enable = 0 (the default) uses the H pass and the E pass.  Other blocks
 * always take the two passes.  Both give the same fields up to rounding. */
sbp_status sbp_set_fused(sbp_ctx *ctx, int enable, int planes);

/* Measures candidate launch shapes on the current state (restored after)
 * and keeps the fastest; writes ms per step of the winner. */
sbp_status sbp_autotune(sbp_ctx *ctx, int steps_per_trial, double *best_ms);

/* Records `steps` consecutive steps in a HIP graph; later sbp_step calls
 * replay it for whole multiples of `steps` (0 disables). */
sbp_status sbp_use_graph(sbp_ctx *ctx, int steps);

/* Time (ms) of the last sbp_step call between HIP events on the stream;
 * valid after the stream has reached the end event. */
sbp_status sbp_last_step_ms(sbp_ctx *ctx, double *ms);

/* Mean time (ms) per step of the H pass, the E pass and the one-pass
 * launches over the last sbp_step call, from HIP events around each group of
 * launches on the context's stream (enabled by sbp_profile(ctx,1)). */
sbp_status sbp_profile(sbp_ctx *ctx, int enable);
sbp_status sbp_kernel_ms(sbp_ctx *ctx, double out[3]);

const char *sbp_last_error(const sbp_ctx *ctx);
void sbp_destroy(sbp_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
