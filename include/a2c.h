/*
 * a2c.h -- C ABI of the MI355X (gfx950) library that maps protein dihedral
 * angles to atomic Cartesian coordinates and maps coordinate gradients back
 * to angle gradients.
 *
 * Method: Derevyanko & Lamoureux, "TorchProteinLibrary: A computationally
 * efficient, differentiable representation of protein structure",
 * arXiv:1812.01108.
 *   - backbone model ("Backbone model" section): per residue j three
 *     transforms R(omega_j), R(phi_j), R(psi_j) place N_j, CA_j, C_j;
 *     r_i = R_0 R_1 ... R_i 0; gradient = the sums of Eq. BackboneGradOutput;
 *   - full-atom model ("Full-atom model" section): a graph of transforms
 *     M_i = M_parent(i) R_i acting on standard rigid-group coordinates r°,
 *     up to 7 dihedrals per residue (phi, psi, omega, chi1..chi4); gradient
 *     = Eq. FAMBackward;
 *   - every transform is R(alpha, theta, d) = Ry(theta) Tx(d) Rx(alpha)
 *     with the 4x4 matrix printed in the backbone section.
 *
 * Conventions shared by every call
 *   - Pointers prefixed d_ are device pointers (hipMalloc'ed or torch CUDA
 *     tensors); h_ pointers are host memory.  The caller owns every device
 *     buffer.  The library owns only the plan and the device copies of the
 *     plan's tables, freed by a2c_plan_destroy.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     a2c_forward, a2c_backward, a2c_mse_step, a2c_lrmsd_forward,
 *     a2c_lrmsd_backward and a2c_coords_to_angles only enqueue kernels on
 *     it: they never allocate, never synchronise and never read device
 *     memory on the host, so they may be captured in a hipGraph (replays
 *     reproduce the eager results bit for bit).  Plan creation, schedule
 *     changes and autotuning upload tables and synchronise: not capturable.
 *   - Angles are radians, any range; NaN/Inf propagate unchecked.  Planes:
 *       0 phi, 1 psi, 2 omega, 3 chi1, 4 chi2, 5 chi3, 6 chi4.
 *     Layout [K][R] float32, K = 3 (backbone) or 7 (full-atom), R = total
 *     residues over all chains (chains packed back to back).
 *   - Coordinates: layout [3][A] float32 (x plane, y plane, z plane), A =
 *     total atoms.  Backbone: atoms 3j, 3j+1, 3j+2 of residue j are N, CA, C.
 *     Full-atom: per residue N, CA, C, O, then side-chain atoms in the order
 *     of the residue table; chain and residue atom offsets come from the plan.
 *   - Each chain starts from the identity frame: its first N sits at
 *     (d cos theta, 0, -d sin theta) of the C-N bond transform.
 *   - Errors are returned, never raised; validation is host-side and happens
 *     before anything is enqueued.  a2c_last_error() gives a thread-local
 *     message for the last failing call.
 *   - A plan is not safe for concurrent calls from several threads.
 */
#ifndef A2C_H
#define A2C_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    A2C_OK = 0,
    A2C_ERR_INVALID_ARG = -1,  /* bad pointer, size, offset or residue code  */
    A2C_ERR_UNSUPPORTED = -2,  /* valid input the chosen schedule cannot run */
    A2C_ERR_WORKSPACE = -3,    /* workspace missing or too small             */
    A2C_ERR_HIP = -4,          /* a HIP runtime call failed                  */
    A2C_ERR_STATE = -5         /* call out of order (e.g. no device)         */
} a2c_status;

/* Selector arguments (model, variant, a status to describe) are passed as
 * int32_t holding one of these values, so that any other value is refused
 * with A2C_ERR_INVALID_ARG (or described as unknown) rather than being an
 * out-of-range enumeration value. */
typedef enum { A2C_BACKBONE = 0, A2C_FULLATOM = 1 } a2c_model;

/* A2C_SCAN: the library's form -- segmented scans over 3x4 affine transforms
 *   in registers, whole chains packed into workgroup tiles, O(N) adjoint.
 * A2C_PLAIN: the paper's GPU design kept as a comparison (backbone only):
 *   one workgroup per chain, a sequential transform product that stores M_i
 *   for every atom, and the O(atoms x angles) gradient sum of
 *   Eq. BackboneGradOutput.  Needs a workspace (a2c_plan_workspace_bytes). */
/* A2C_SCAN_QUAT: the scan form with a different scan state, kept as a
 *   measured comparison (backbone a2c_forward only; a2c_backward refuses it
 *   with A2C_ERR_UNSUPPORTED): the state the scans and the window look-back
 *   combine is a unit quaternion and a translation (7 floats, the quaternion
 *   form of the transforms in the "Loss function" section) instead of the
 *   3x4 affine.  The lane walk is the same; each lane aggregate, after its
 *   polar step, is converted (Shepperd's method, normalised) and the lane's
 *   prefix is converted back to place its atoms.  In float32 the rotation a
 *   quaternion holds carries a larger rounding error that similar residues
 *   repeat: at L = 1000 its coordinates drift further (8.2e-4 A against
 *   5.8e-4 A for A2C_SCAN on 64 mixture chains, 8 residues per lane), too
 *   close to the 1e-3 A bound for a forward only a few percent faster; the
 *   library's results use A2C_SCAN. */
typedef enum { A2C_SCAN = 0, A2C_PLAIN = 1, A2C_SCAN_QUAT = 2 } a2c_variant;

typedef struct a2c_plan a2c_plan;

/* Backbone geometry, named by bonded atoms and by the vertex of each angle.
 * The transform placing N_j uses bond C-N and theta = pi - angle(CA-C-N);
 * the one placing CA_j uses N-CA and pi - angle(C-N-CA); the one placing C_j
 * uses CA-C and pi - angle(N-CA-C).  Lengths in Angstrom, angles in degrees.
 * NULL where a geometry is accepted means: 1.458, 1.525, 1.329 A and
 * 111.2, 116.2, 121.7 degrees. */
typedef struct {
    double bond_n_ca, bond_ca_c, bond_c_n;
    double angle_n_ca_c, angle_ca_c_n, angle_c_n_ca;
} a2c_backbone_geometry;

/* ---- full-atom residue table ------------------------------------------ *
 * The paper's per-residue graph: spine frames 0 (N, placed by omega),
 * 1 (CA, by phi), 2 (C, by psi) use the backbone geometry; side-chain frames
 * 3..6 hang off CA or off an earlier side frame.  Each residue type lists
 * its atoms in output order with the frame they belong to and their
 * standard position r° in that frame, given as internal coordinates that
 * the library converts to Cartesian r° at plan creation.               */
#define A2C_NUM_RESIDUE_TYPES 20
#define A2C_MAX_SIDE_FRAMES 4
#define A2C_MAX_RESIDUE_ATOMS 14

typedef struct {
    int32_t parent;            /* 1 = CA frame, 3.. = earlier side frame      */
    int32_t chi;               /* 1..4: torsion is chi_k (plane 2+k); 0: fixed 0 */
    double pre_rotation_deg;   /* fixed rotation about the parent's x axis
                                  applied before the transform (R' of the
                                  threonine example); 0 for none           */
    double bond;               /* parent origin atom -> this origin atom (A)  */
    double bond_angle_deg;     /* angle (parent's predecessor, parent origin,
                                  this origin)                               */
} a2c_side_frame;

/* Atom kinds: */
#define A2C_ATOM_ORIGIN 0      /* at the frame origin                          */
#define A2C_ATOM_AZIMUTH 1     /* bonded to the frame origin: length `bond`,
                                  angle (predecessor, origin, atom) = `angle`,
                                  torsion = frame torsion + `torsion`          */
#define A2C_ATOM_ZMATRIX 2     /* from atoms ref[0..2] of the same frame (-1 =
                                  the frame's predecessor atom): |ref2 - a| =
                                  bond, angle(ref1, ref2, a) = angle,
                                  torsion(ref0, ref1, ref2, a) = torsion      */
typedef struct {
    int32_t frame;             /* 0 N, 1 CA, 2 C, 3 + f = side frame f        */
    int32_t kind;              /* A2C_ATOM_*                                   */
    int32_t ref[3];            /* atom indices within the residue, or -1      */
    double bond, angle_deg, torsion_deg;
} a2c_atom_def;

typedef struct {
    int32_t n_atoms;           /* heavy atoms incl. N, CA, C, O (<= 14)        */
    int32_t n_side_frames;     /* 0 .. 4                                        */
    a2c_side_frame frames[A2C_MAX_SIDE_FRAMES];
    a2c_atom_def atoms[A2C_MAX_RESIDUE_ATOMS];
} a2c_residue_def;

typedef struct {
    a2c_residue_def residues[A2C_NUM_RESIDUE_TYPES];
} a2c_residue_table;

/* Create a plan for one packed batch of chains (the paper's statement of the
 * problem: angles and, for the full-atom model, the residue sequence, since
 * theta and d depend only on the residue type; "Full-atom model" section).
 *   h_res_offsets  host int32[n_chains + 1]: [0] = 0, non-decreasing, last =
 *                  R.  Zero-length chains are allowed and produce nothing.
 *   h_seq          host uint8[R] residue codes 0..19 (table order); required
 *                  for A2C_FULLATOM, ignored (may be NULL) for A2C_BACKBONE.
 *   geom           backbone geometry or NULL for the defaults above.
 *   table          residue table, required for A2C_FULLATOM.
 *   mem_budget_bytes  store-vs-recompute threshold for the memory kept
 *                  between the forward and the adjoint: the forward's
 *                  coordinates (12 bytes per atom) are worth keeping for the
 *                  adjoint while they fit in it (a2c_plan_keep_coords); 0 =
 *                  always recompute the frames from the angles in the
 *                  adjoint; SIZE_MAX = no limit.  Per-atom transforms are
 *                  never stored by the scan form.
 *   stream         used for the table uploads; the call synchronises it.
 * Picks a default schedule (a2c_plan_set_schedule) that runs the longest
 * chain.  Fails with A2C_ERR_INVALID_ARG on malformed offsets or codes >= 20,
 * and with A2C_ERR_UNSUPPORTED, before any device call, if a chain is longer
 * than 64 chunks of the widest schedule (262144 residues for A2C_BACKBONE,
 * 131072 for A2C_FULLATOM), or if the full-atom default schedule cannot stage
 * its atoms in LDS.  *out is NULL on failure.                             */
a2c_status a2c_plan_create(a2c_plan **out, int32_t model, int32_t n_chains,
                           const int32_t *h_res_offsets, const uint8_t *h_seq,
                           const a2c_backbone_geometry *geom,
                           const a2c_residue_table *table, size_t mem_budget_bytes,
                           void *stream);

/* The plan's store-vs-recompute choice: *keep = 1 when the forward's
 * coordinates (12 bytes per atom, A atoms) fit the plan's memory budget, so
 * a2c_backward should be given them (d_coords); 0 when the adjoint should
 * recompute the frames from the angles (d_coords = NULL).  Host only.  Both
 * choices give the same gradient up to float32 rounding. */
a2c_status a2c_plan_keep_coords(const a2c_plan *plan, int32_t *keep);

void a2c_plan_destroy(a2c_plan *plan);

/* Total residues R and atoms A of the plan.  (The workspace size a variant
 * needs is a2c_plan_workspace_bytes.) */
a2c_status a2c_plan_sizes(const a2c_plan *plan, int64_t *n_res, int64_t *n_atoms);

/* Atom offsets: h_chain_atom_offsets int32[n_chains + 1] (may be NULL),
 * h_res_atom_offsets int32[R + 1] (may be NULL). */
a2c_status a2c_plan_atom_offsets(const a2c_plan *plan, int32_t *h_chain_atom_offsets,
                                 int32_t *h_res_atom_offsets);

/* Device workspace a variant needs (0 for A2C_SCAN; 48 bytes per atom for
 * A2C_PLAIN, which stores M_i for every atom as the paper's forward does). */
a2c_status a2c_plan_workspace_bytes(const a2c_plan *plan, int32_t variant,
                                    size_t *bytes);

/* Scan schedule: residues per lane (1, 2 or 4 for A2C_BACKBONE; 1 or 2 for
 * A2C_FULLATOM) and waves of 64 lanes per workgroup (1..16).  A chunk is
 * 64 * waves * res_per_lane consecutive residues.
 *   - The forwards of both models (a2c_forward, A2C_SCAN), the backbone
 *     adjoint from coordinates (a2c_backward with d_coords) and every
 *     full-atom adjoint (a2c_backward, a2c_mse_step) run on windows:
 *     workgroup t takes residues [s_t, s_t+1) of the packed batch, at most
 *     one chunk C.  Where every chain fits in one chunk, the windows hold
 *     whole chains, packed in order; otherwise they are fixed,
 *     [t C, t C + C), whatever the chain boundaries.  A chain entering a
 *     window from earlier ones gets its frame from those windows' aggregates
 *     (forward), and a chain running on into later windows gets their
 *     wrench sums (adjoint); every workgroup publishes its own in plan-owned
 *     device memory before it reads any (window look-back), and waits only
 *     on workgroups started before it or at most 7 places after it (the
 *     adjoints take fixed windows last to first, in each class of workgroup
 *     index mod 8 separately, and whole-chain ones in order; the full-atom
 *     ones that recompute the frames first run a spine-only pass over the
 *     same windows, which waits on nothing); a launch therefore progresses
 *     whenever the device holds 8 of its workgroups at once.  Consequently
 *     two such calls on one plan must not run at the same time (on
 *     different streams).
 *   - The backbone adjoint that recomputes the frames (a2c_backward without
 *     d_coords) and the backbone a2c_mse_step pack chains of at most one
 *     chunk whole, in order, into tiles of at most one chunk; a longer chain
 *     gets a tile of its own, which one workgroup walks chunk by chunk (at
 *     most 64 chunks), carrying the frame (forward) and the wrench (adjoint)
 *     from chunk to chunk.  One workgroup per tile, longest tiles dispatched
 *     first.
 * Re-packs and re-uploads the tables (synchronises `stream`).
 * The tables of the schedule it replaces stay allocated until
 * a2c_plan_destroy, so a graph captured before the change replays the
 * schedule it captured, with the same results; no graph captured over a plan
 * may be replayed after the plan is destroyed.
 * UNSUPPORTED, leaving the plan's schedule as it was, if the longest chain
 * needs more than 64 chunks.  Full-atom atom I/O goes through a per-wave LDS
 * stage (three float planes; the adjoint from coordinates stages six and
 * recomputes the frames from the angles instead where those do not fit,
 * with the same result); where the waves' atoms of one chunk exceed 136 KiB
 * of LDS, the kernels read and write atoms in global memory directly. */
a2c_status a2c_plan_set_schedule(a2c_plan *plan, int32_t res_per_lane,
                                 int32_t waves_per_group, void *stream);
a2c_status a2c_plan_get_schedule(const a2c_plan *plan, int32_t *res_per_lane,
                                 int32_t *waves_per_group, int32_t *n_tiles);

/* A plan holds two schedules with their own tables: the forward's
 * (a2c_forward) and the adjoint's (a2c_backward and a2c_mse_step); the two
 * kernels favour different shapes (more residues per lane suits the forward
 * scan, fewer the adjoint's larger per-lane state).  a2c_plan_set_schedule
 * sets both and a2c_plan_get_schedule reports the forward's; the calls below
 * set or report one of them alone (same arguments, checks and
 * synchronisation as a2c_plan_set_schedule; on failure that schedule is
 * unchanged), except that the backbone forward also takes 8 residues per
 * lane.  Results do not depend on the schedules beyond float32 rounding. */
a2c_status a2c_plan_set_forward_schedule(a2c_plan *plan, int32_t res_per_lane,
                                         int32_t waves_per_group, void *stream);
a2c_status a2c_plan_set_adjoint_schedule(a2c_plan *plan, int32_t res_per_lane,
                                         int32_t waves_per_group, void *stream);
a2c_status a2c_plan_get_adjoint_schedule(const a2c_plan *plan, int32_t *res_per_lane,
                                         int32_t *waves_per_group, int32_t *n_tiles);

/* Autotuner: times the forward (A2C_SCAN) under every schedule
 * a2c_plan_set_forward_schedule accepts for the plan and keeps the fastest,
 * then the adjoint under every schedule a2c_plan_set_adjoint_schedule
 * accepts, on the caller's buffers (candidates in order of residues per
 * lane, then waves; a later one must be 1 % faster than the best so far to
 * replace it, so ties resolve to the smaller schedule).
 *   d_angles, d_coords, d_grad_coords, d_grad_angles: buffers of the plan's
 *     sizes; their contents are overwritten (coords and grad_angles) or read.
 *   backward_from_coords: the adjoint timed: 1 a2c_backward with d_coords
 *     (the forward's output), 0 the recompute form, A2C_TUNE_MSE_STEP the
 *     fused step a2c_mse_step with d_grad_coords as its target.
 *   reps: timed repetitions per candidate (>= 1).
 *   cache_path: text file of earlier choices, keyed by device name, model,
 *     residue count, longest chain, chain count and the adjoint timed
 *     (coords, recompute or mse); NULL for none.  A line is
 *     "<key> K W aK aW" (or "<key> K W" for both).  A hit skips the timing;
 *     a miss appends the new choice.  An unreadable cache, and any line that
 *     is malformed or names schedules the forward or adjoint setter would
 *     reject for the plan, are ignored (the schedules are then tuned).
 *   out_res_per_lane, out_waves_per_group (may be NULL): the forward's
 *     choice (a2c_plan_get_adjoint_schedule gives the adjoint's).
 * Synchronises `stream`; not capturable.  Call it before capturing a graph. */
#define A2C_TUNE_MSE_STEP 2
a2c_status a2c_plan_autotune(a2c_plan *plan, const float *d_angles, float *d_coords,
                             const float *d_grad_coords, float *d_grad_angles,
                             int32_t backward_from_coords, int32_t reps, const char *cache_path,
                             int32_t *out_res_per_lane, int32_t *out_waves_per_group,
                             void *stream);

/* Forward map: d_angles [K][R] -> d_coords [3][A].
 * d_workspace: NULL for A2C_SCAN; for A2C_PLAIN a buffer of
 * a2c_plan_workspace_bytes that a2c_backward(A2C_PLAIN) reads later. */
a2c_status a2c_forward(a2c_plan *plan, int32_t variant, const float *d_angles,
                       float *d_coords, void *d_workspace, void *stream);

/* Adjoint: given d_grad_coords = dL/dr [3][A], writes dL/dalpha [K][R]
 * (every plane; chi planes a residue lacks are written as 0).
 *   d_coords   the coordinates a2c_forward produced from the same angles, or
 *              NULL: A2C_SCAN then recomputes the frames from the angles
 *              inside the backward kernel (nothing is stored between the two
 *              passes).  A2C_PLAIN requires the workspace its forward filled.
 * The result is exact up to float32 rounding: for angle alpha_i of node i,
 *   dL/dalpha_i = u_i . sum_{k in subtree(i)} (r_k - r_i) x dL/dr_k,
 * u_i the unit bond vector the node rotates about, which equals the sums of
 * Eq. BackboneGradOutput / Eq. FAMBackward.
 * The adjoint on windows writes d_grad_angles with non-temporal stores when
 * it holds at least 4 MiB (the plan's R x K floats): the caches then keep the
 * step's coordinates and upstream gradients instead.  The values are the
 * same either way. */
a2c_status a2c_backward(a2c_plan *plan, int32_t variant, const float *d_angles,
                        const float *d_coords, const float *d_grad_coords,
                        float *d_grad_angles, void *d_workspace, void *stream);

/* Inverse map: coordinates [3][A] in the plan's layout -> angles [K][R],
 * the step before the forward map in a pipeline (targets, initial angles).
 * The angle of the transform placing atom i is the IUPAC torsion about the
 * bond into atom i ("Backbone model" section), so
 *   omega_j = torsion(CA_{j-1}, C_{j-1}, N_j, CA_j),
 *   phi_j   = torsion(C_{j-1}, N_j, CA_j, C_j),
 *   psi_j   = torsion(N_j, CA_j, C_j, N_{j+1}),
 * in (-pi, pi]; at a chain start the start frame's virtual atoms
 * C_{-1} = origin and CA_{-1} = (-1, 0, 0) stand in (so omega_0 and phi_0
 * also fix the chain's orientation in that frame); psi of a chain's last
 * residue moves no atom and is written as 0.  Full-atom plans also write
 * chi1..chi4 (the torsion carried by each side frame, equal to the IUPAC
 * chi of the residue table) and 0 in planes a residue lacks.  Forward then
 * inverse returns the input angles up to float32 rounding (and psi of last
 * residues).  One kernel on `stream`, no allocation (capturable). */
a2c_status a2c_coords_to_angles(a2c_plan *plan, const float *d_coords, float *d_angles,
                                void *stream);

/* Fused training step for the squared-distance loss
 *   L = sum over atoms a of |r_a - t_a|^2
 * (r the map of d_angles, t = d_target [3][A]): one kernel, one workgroup
 * per tile, recomputes the frames, forms the loss gradient 2 (r - t) in
 * registers and runs the adjoint above, so neither the coordinates nor
 * their gradient make a round trip through memory.  Same result as
 * a2c_forward, then dL/dr = 2 (r - t), then a2c_backward, up to float32
 * rounding.
 *   d_coords      [3][A] receives r, or NULL (not written);
 *   d_loss        float[1] receives L, or NULL (not computed).  Each tile
 *                 adds its atoms in a fixed order into a share kept in the
 *                 plan; the tile that finishes last sums the shares in tile
 *                 order, so L is deterministic for a given schedule.
 *   d_grad_angles [K][R] receives dL/dalpha.
 * Enqueues one kernel on `stream` (a fill kernel for an empty plan); no
 * allocation (capturable).  Calls that share a plan must not overlap. */
a2c_status a2c_mse_step(a2c_plan *plan, const float *d_angles, const float *d_target,
                        float *d_coords, float *d_loss, float *d_grad_angles, void *stream);

/* ----------------------------------------------------------------- LRMSD
 * The loss the paper pairs with the map (section "Loss function"): for each
 * chain c of the plan, with x the target and y the input coordinates of its
 * N atoms, x~ and y~ the sets centred on their means and
 * R = sum_i x~_i y~_i^T,
 *   LRMSD_c = min over rigid motions of the root-mean-square deviation
 *           = sqrt((sum |x~|^2 + sum |y~|^2 - 2 lambda) / N),
 * lambda the largest eigenvalue of the section's 4x4 matrix T(R), q its unit
 * eigenvector and U(q) the section's rotation, which maps the target onto
 * the input (U x~_i ~ y~_i).  The gradient with respect to the input is
 *   dLRMSD_c / dy_i = (y~_i - U x~_i) / (N LRMSD_c),
 * taken as 0 for a chain with LRMSD_c = 0 or no atoms.  (The section prints
 * the derivative with respect to the target without the 1 / (N LRMSD)
 * factor.)  Sums are accumulated in float64; at a repeated largest
 * eigenvalue U is one of the optimal rotations and the gradient is not
 * unique.
 *
 * Workspace: a device buffer of a2c_lrmsd_workspace_bytes, owned by the
 * caller; a2c_lrmsd_forward fills it (per-chain U, means and 1 / (N LRMSD))
 * and a2c_lrmsd_backward reads it, so the backward needs the same buffer,
 * untouched, and the same coordinates and target. */
a2c_status a2c_lrmsd_workspace_bytes(const a2c_plan *plan, size_t *bytes);

/* d_coords, d_target: [3][A] float32 planes (the plan's atom layout);
 * d_lrmsd: float32[n_chains] per-chain LRMSD.  Two kernels on `stream`, no
 * allocation, no synchronisation (capturable). */
a2c_status a2c_lrmsd_forward(a2c_plan *plan, const float *d_coords, const float *d_target,
                             float *d_lrmsd, void *d_workspace, void *stream);

/* d_grad_lrmsd: float32[n_chains] upstream gradient of each LRMSD_c;
 * writes d_grad_coords [3][A] = sum_c d_grad_lrmsd[c] dLRMSD_c / dy (zero for
 * atoms of empty or zero-LRMSD chains).  One kernel on `stream`. */
a2c_status a2c_lrmsd_backward(a2c_plan *plan, const float *d_coords, const float *d_target,
                              const float *d_grad_lrmsd, float *d_grad_coords,
                              const void *d_workspace, void *stream);

/* No-allocation form of a2c_lrmsd_forward, for callers that cannot allocate
 * device memory: code under graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments (without the workspace), kernels
 * and results (bit for bit) as a2c_lrmsd_forward; the segment sums and
 * per-chain state go to a fixed array of A2C_LRMSD_STATIC_BYTES (4 MiB)
 * that the library holds on every device it runs on, from module load until
 * the process ends, instead of a caller's workspace.  Allocates and frees
 * nothing; its device address is taken when a plan is created on that
 * device.
 *   Fails with A2C_ERR_WORKSPACE, before anything is enqueued, when the plan
 *   needs more (a2c_lrmsd_workspace_bytes > A2C_LRMSD_STATIC_BYTES: 144
 *   bytes per segment of up to 4096 atoms of one chain plus 64 per chain,
 *   e.g. about 20 000 short chains or 28 000 segments).
 *   Every call on a device shares that device's array and leaves its
 *   contents there: calls that overlap on one device (several streams or
 *   threads) race and give wrong results.  a2c_lrmsd_backward takes a
 *   caller's workspace, never this array.
 * Two kernels on `stream`, no synchronisation (capturable). */
#define A2C_LRMSD_STATIC_BYTES (4u << 20)
a2c_status a2c_lrmsd_forward_noalloc(a2c_plan *plan, const float *d_coords,
                                     const float *d_target, float *d_lrmsd, void *stream);

/* Host-only check of a residue table (no device needed): validates it as
 * a2c_plan_create would and reports, per residue type, the atom count
 * (n_atoms int32[20], may be NULL) and the standard position r° of every
 * atom in its own frame (local_xyz float[20][14][3] by output slot, may be
 * NULL), as the library derives them from the internal coordinates.
 * Spine-frame predecessor distances use the default backbone geometry.
 * Constraints beyond the struct's own: atoms 0, 1, 2 are N, CA, C at the
 * spine frame origins; side frame 0 hangs off CA (only it may have a
 * pre-rotation), side frame f > 0 off side frame f - 1 with chi = f + 1 or
 * 0; every frame has exactly one atom at its origin; z-matrix references
 * are earlier atoms of the same frame or the frame's predecessor. */
a2c_status a2c_residue_table_info(const a2c_residue_table *table, int32_t *n_atoms,
                                  float *local_xyz);

const char *a2c_status_string(int32_t status);
const char *a2c_last_error(void);

/* Library version string, e.g. "a2c 0.1 gfx950". */
const char *a2c_version(void);

#ifdef __cplusplus
}
#endif

#endif /* A2C_H */
