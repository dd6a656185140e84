/*
 * cylpoisson -- full-spectrum cylindrical Poisson solve on one AMD Instinct
 * MI355X (gfx950): azimuthal DFT, batched matrix-free geometric multigrid on
 * every Fourier plane, inverse DFT.
 *
 * The equation is the cylindrical Poisson equation of Sec. 3.1,
 *     -[ (1/r) d/dr (r dphi/dr) + (1/r^2) d2phi/dtheta^2 + d2phi/dz^2 ] = rho/eps0,
 * discretised by the finite-volume cell balance of App. A on an annular
 * tensor-product mesh (vertex-centred, or cell-centred with half-cell
 * Dirichlet faces, uniform or not in r and z), with the periodic three-point
 * azimuthal difference of Sec. 3.1.  The solve follows Sec. 3: the azimuthal DFT (Eq. azimuthal_dft)
 * splits the 3-D system into independent 2-D systems A_m = A_0 + lambda_m M
 * (Eq. shifted_operator_family) with the exact discrete eigenvalue
 * lambda_m = (4/dtheta^2) sin^2(pi m / Ntheta) (Eq. discrete_azimuthal_eigenvalue),
 * right-hand side s_q rho^_m + b^D delta_{m0} (Eq. mode_rhs); every mode is
 * solved by V-cycles over one shared hierarchy, and the inverse DFT returns phi.
 *
 * Conventions
 * -----------
 * Grid.  Nr radial and Nz axial nodes, both counts including the two
 *   Dirichlet nodes of the direction; Ntheta periodic nodes
 *   theta_j = 2 pi j / Ntheta over the full annulus.  cylpoisson_plan_create
 *   builds the uniform vertex-centred mesh r_i = r_in + i (r_out - r_in)/(Nr - 1),
 *   z_k = k dz; cylpoisson_plan_create_mesh takes explicit coordinates.
 * Arrays.  Node arrays are C-contiguous double[Ntheta][Nz][Nr] (r fastest) in
 *   device memory of the plan's device.  rho in C/m^3, phi in volts,
 *   eps0 = 8.8541878128e-12 F/m.
 * Planes.  The N = Ntheta real planes of a node array x are
 *     plane m          (m = 0 .. floor(N/2))      : Re x^_m
 *     plane floor(N/2)+m (m = 1 .. ceil(N/2) - 1) : Im x^_m
 *   with x^_m = (1/N) sum_j x_j exp(-2 pi i m j / N) (Eq. azimuthal_dft).
 *   Plane arrays have the node-array shape; plane p replaces azimuthal index p.
 * Ownership.  All pointers passed in are owned by the caller; the plan owns
 *   its device workspace from create to destroy.
 * Streams.  `stream` is a hipStream_t (NULL = default stream) of the plan's
 *   device.  Every kernel is enqueued on it.  Calls that need a convergence
 *   decision synchronise that stream.  A plan runs one call at a time; calls
 *   on different plans may run concurrently.
 * Errors.  Functions return a status (below); on failure a thread-local
 *   message is available from cylpoisson_last_error().  Arguments are
 *   validated before any device work is enqueued.
 */
#ifndef CYLPOISSON_H
#define CYLPOISSON_H

#ifdef __cplusplus
extern "C" {
#endif

#define CYLPOISSON_OK 0
#define CYLPOISSON_NOT_CONVERGED 1 /* tolerance not reached; phi holds the last iterate */
#define CYLPOISSON_EINVAL (-1)     /* invalid argument */
#define CYLPOISSON_ENOMEM (-2)     /* device or host allocation failed */
#define CYLPOISSON_EHIP (-3)       /* a HIP runtime call failed */
#define CYLPOISSON_ENONFINITE (-4) /* rho (or a plane right-hand side) holds NaN or Inf */
#define CYLPOISSON_EDEVICE (-5)    /* a pointer is not device memory of the plan's device */

/* Mesh layouts of cylpoisson_plan_create_mesh (App. A). */
#define CYLPOISSON_VERTEX 0 /* unknowns at the given nodes, control-volume faces half-way */
#define CYLPOISSON_CELL 1   /* unknowns at cell centres, Dirichlet values on the outer faces */

#define CYLPOISSON_MAX_HISTORY 64
#define CYLPOISSON_MAX_LEVELS 24
#define CYLPOISSON_KERNEL_CLASSES 7

typedef struct cylpoisson_plan cylpoisson_plan; /* opaque */
typedef struct cylpoisson_nn cylpoisson_nn;     /* opaque: the learned preconditioner's network */

/* Dirichlet values (volts) on the four faces, invariant in theta, so that only
 * the m = 0 mode carries a boundary term (Eq. mode_rhs).  The axial faces win
 * at the (r, z) corners. */
typedef struct {
    double phi_r_in, phi_r_out, phi_z0, phi_zL;
} cylpoisson_bc;

typedef struct {
    int status;          /* status returned by the last solve */
    int cycles;          /* V-cycles performed by the last solve */
    int checks;          /* host convergence checks (stream synchronisations) */
    int n_history;       /* entries of rel_residual_history that are set */
    double rel_residual; /* final relative residual (definition below) */
    double initial_residual_norm; /* ||b|| in finite-volume scaling */
    /* relative residual after cycle c (index c - 1); NaN where not evaluated
     * (cycles that end in a merged finest pass, option "merge").
     * Relative residual = sqrt(sum_p w_p ||r_p||^2 / sum_p w_p ||b_p||^2) over
     * interior nodes, with the Parseval weights w_p = 1 for m = 0 and m = N/2,
     * 2 otherwise, i.e. the 2-norm of the 3-D residual relative to that of the
     * 3-D right-hand side s rho + b^D. */
    double rel_residual_history[CYLPOISSON_MAX_HISTORY];
    /* Device time per kernel class in the last solve, from HIP events recorded
     * around each launch on the solve's stream when the option "timing" is 1,
     * for classes 2, 3 and 6 only when it is 2 (all zero otherwise).  Classes: 0 forward DFT, 1 inverse DFT, 2 finest-level
     * down pass (smoothing, residual, restriction), 3 finest-level up pass
     * (prolongation, smoothing, residual norm), 4 all coarser levels (one
     * interval per cycle), 5 other work (initialisation, norm reductions, the
     * FP64 refinement steps of a mixed-precision solve), 6 finest-level merged
     * pass (the up pass of one cycle and the down pass of the next, option
     * "merge"). */
    int kernel_launches[CYLPOISSON_KERNEL_CLASSES];
    double kernel_ms[CYLPOISSON_KERNEL_CLASSES];
    /* Mixed precision ("precision" = 32): FP64 refinement steps after the
     * first residual, i.e. the number of FP32 inner solves; `cycles` counts
     * their FP32 V-cycles and the history holds the FP64 relative residual
     * after each inner solve (at index cycles - 1).  0 on the FP64 path. */
    int refinements;
    /* Planes frozen by the option "masks" when the solve ended (0 otherwise). */
    int frozen_planes;
    /* Learned solve (option "krylov" = 1): FGMRES steps taken, the relative
     * residual after the judging V-cycle (its contraction from zero), the
     * network's mean contraction per FGMRES step over the judged restart, and
     * 1 if V-cycles finished the solve because the network contracted less. */
    int krylov_iterations;
    int learned_fallback;
    double vcycle_rate;
    double learned_rate;
} cylpoisson_stats;

typedef struct {
    int nr, ntheta, nz;
    int levels;                             /* multigrid levels (1 = direct only) */
    int level_nr[CYLPOISSON_MAX_LEVELS];    /* nodes per level, incl. the ring */
    int level_nz[CYLPOISSON_MAX_LEVELS];
    int coarse_unknowns;                    /* interior nodes of the coarsest plane */
    int bottom_level;                       /* first level run by the LDS bottom kernel, -1 if none */
    long long workspace_bytes;              /* device memory owned by the plan */
    int device;                             /* HIP device ordinal */
    int fused_levels;   /* levels from the finest whose V-cycle work runs in fused streaming
                         * passes under the current options (the others above the bottom
                         * kernel run one kernel per sweep) */
    int layout;         /* CYLPOISSON_VERTEX or CYLPOISSON_CELL */
    int uniform;        /* 1 = built by cylpoisson_plan_create (uniform vertex-centred mesh) */
    int direct_level;   /* level solved exactly by the separable solve, where the V-cycle
                         * stops under the current option "direct"; -1 if none or off */
} cylpoisson_info;

/* Create a plan for an Nr x Ntheta x Nz grid.  Requires Nr >= 3, Nz >= 3,
 * Ntheta >= 1, 0 < r_in < r_out, dz > 0 and finite boundary values.  Builds
 * the multigrid hierarchy and its coefficient tables on the host, allocates
 * the device workspace on the current HIP device and uploads the tables.
 * Returns NULL on error (cylpoisson_last_status: EINVAL, ENOMEM or EHIP;
 * cylpoisson_last_error describes it). */
cylpoisson_plan* cylpoisson_plan_create(int Nr, int Ntheta, int Nz, double r_in, double r_out,
                                        double dz, const cylpoisson_bc* bc);

/* Create a plan on an explicit, possibly non-uniform mesh (App. A: the cell
 * balance with conductances from the actual face positions and node
 * distances).  r and z are host arrays, read during the call only.
 *   layout CYLPOISSON_VERTEX: r holds the Nr node radii and z the Nz node
 *     heights, boundary nodes included; the control volume of an interior node
 *     reaches half-way to each neighbour.
 *   layout CYLPOISSON_CELL: r holds the Nr - 1 radial faces of the Nr - 2
 *     cells and z the Nz - 1 axial faces of the Nz - 2 cells.  The unknowns sit
 *     at the cell centres (face midpoints); the outer faces are the Dirichlet
 *     nodes, half a cell from the first centre, which gives the half-cell
 *     boundary conductance of Eq. (dirichlet_face_conductances).
 * In both layouts node arrays keep the shape [Ntheta][Nz][Nr]: the ring holds
 * the Dirichlet values, the interior the unknowns.  Requires Nr, Nz >= 3,
 * Ntheta >= 1, finite strictly increasing coordinates, r[0] > 0, finite
 * boundary values.  Coarser multigrid levels keep every other node of each
 * coarsened direction and rediscretise with faces half-way between their
 * nodes; grid transfers interpolate linearly in the coordinates, and a
 * direction is coarsened alone while the median spacings differ more than
 * 2:1.  Returns NULL on error (cylpoisson_last_status: EINVAL, ENOMEM or EHIP). */
cylpoisson_plan* cylpoisson_plan_create_mesh(int Nr, int Ntheta, int Nz, const double* r, const double* z,
                                             int layout, const cylpoisson_bc* bc);

/* Release the plan and its device memory.  NULL-safe.  The plan must be idle. */
void cylpoisson_plan_destroy(cylpoisson_plan* plan);

/* Set a solver option.  Keys (value ranges):
 *   "nu1", "nu2"     pre-/post-smoothing sweeps (1 .. 8; default 2, 2)
 *   "nu1_coarse", "nu2_coarse"  the same on every level below the finest
 *                    (0 .. 8; 0 = nu1, nu2; default 0, 0)
 *   "omega"          red-black over-relaxation factor (0 < omega < 2; default 1.15)
 *   "max_cycles"     V-cycle limit per solve (1 .. CYLPOISSON_MAX_HISTORY; default 40)
 *   "check_every"    cycles between host convergence checks once the predicted
 *                    cycle count is reached (1 .. 64; default 1)
 *   "fused"          1 = fused streaming passes (all sweeps, residual and grid
 *                    transfer of a level in one kernel), 0 = one kernel per
 *                    sweep everywhere (default 1)
 *   "chunk_rows"     axial rows per workgroup of the fused passes (0 = automatic)
 *   "prefetch"       rows the fused passes load ahead of the one they consume (1 .. 3; default 1)
 *   "timing"         1 = record per-kernel-class device times (cylpoisson_stats);
 *                    2 = the finest-level pass classes only (fewer event records
 *                    between the other launches); 0 = off (0 .. 2; default 0)
 *   "bottom"         1 = run the small levels of each plane in one LDS-resident
 *                    kernel (with "fused" = 1; default 1)
 *   "smoother"       0 = point red-black SOR (default); 1 = zebra line relaxation
 *                    along r (the interior rows of one parity, then of the other,
 *                    each solved exactly along r with its neighbour rows fixed);
 *                    2 = alternating zebra lines, r-lines then z-lines in every
 *                    sweep, for cells whose aspect ratio varies across the mesh.
 *                    Lines use no over-relaxation and run one kernel per colour,
 *                    so 1 and 2 bypass the fused passes and the LDS bottom kernel
 *                    (and exclude precision 32 and masks, which need them)
 *   "fft"            1 = azimuthal transforms as register FFTs when Ntheta is 16,
 *                    32, 64 or 128; 0 = dense DFT product (default 1)
 *   "precision"      64 = FP64 V-cycles (default); 32 = mixed precision: FP64
 *                    iterative refinement (residual, solution accumulation, DFTs)
 *                    around V-cycles whose smoothing, restriction and prolongation
 *                    run in FP32, with the coarsest solve still in FP64.  Setting
 *                    32 allocates the FP32 level buffers (ENOMEM on failure); it
 *                    needs the fused passes and the LDS bottom kernel on this grid
 *                    (EINVAL otherwise, also at solve time if options changed)
 *   "inner_cycles"   FP32 V-cycles per refinement step (1 .. 8; default 2)
 *   "groups"         plane groups whose V-cycles run on separate streams between
 *                    convergence checks (1 .. 8; default 1; used when every level
 *                    above the bottom kernel has fused passes, else 1).  Results
 *                    do not depend on it
 *   "warm_start"     1 = cylpoisson_solve takes the phi it is given as the initial
 *                    guess (its interior nodes; boundary nodes are ignored and
 *                    rewritten); 0 = zero initial guess, phi not read (default 0)
 *   "masks"          1 = per-plane convergence masks: a plane whose weighted squared
 *                    residual is within tol^2 ||b||^2 / Ntheta stops being cycled
 *                    (its last iterate is kept), FP64 path with fused passes
 *                    (default 0)
 *   "krylov"         1 = learned solve: flexible GMRES with the attached network
 *                    (cylpoisson_plan_set_net) as right preconditioner, judged
 *                    against one plain V-cycle and replaced by V-cycles when it
 *                    contracts less per step (FP64 only; default 0)
 *   "krylov_precond" 1 = the network preconditions FGMRES; 0 = no preconditioner;
 *                    2 = four red-black SOR sweeps, the map the network is trained
 *                    to imitate (0 and 2 for comparison); 3 = one V-cycle from
 *                    zero: multigrid-preconditioned FGMRES, which needs fewer
 *                    steps than plain V-cycles where the point smoother is weak
 *                    (strongly stretched meshes), at one V-cycle plus the Arnoldi
 *                    work per step (counted in `cycles`); not judged (no judging
 *                    cycle, no fallback, vcycle_rate 0) since the plain V-cycle
 *                    iterates lie in the space FGMRES minimises over; 4 = one
 *                    V-cycle from zero followed by the attached network's
 *                    correction of the residual it leaves (z = V(v); z += N(v - A z)):
 *                    the network inside the multigrid preconditioner, judged like 1
 *                    against the plain V-cycle (default 1)
 *   "krylov_restart" FGMRES restart length, also the judged steps (1 .. 16; default 8)
 *   "krylov_max"     FGMRES steps in all (default 200)
 *   "fallback"       1 = V-cycles take over from a worse network (default 1)
 *   "nn_target"      training pairs cylpoisson_nn_collect stores: 0 = each V-cycle
 *                    iterate's residual and the correction four red-black SOR
 *                    sweeps make from it; 1 = the residual after each V-cycle and
 *                    the iterate's error u* - u (u* the solve to tol 1e-14 first)
 *                    (default 0)
 *   "fmg"            1 = full-multigrid start: the right-hand side is restricted
 *                    down to the level where the V-cycle stops, which is solved
 *                    there (exactly under "direct", else by the LDS bottom
 *                    kernel from zero); that answer is interpolated up to level
 *                    1, which takes one V-cycle from it, and the V-cycles on the
 *                    finest level start from the interpolated level-1 answer.
 *                    Its error is then smaller per unit of residual, so a
 *                    looser tol reaches a given error (at 400 x 128 x 512, tol
 *                    1e-13 gives rel-L2 2e-13 in 6 cycles, against 8 cycles
 *                    to 1e-14 from zero).  With "precision" 32 the FP64
 *                    refinement starts from that iterate (its residual measured
 *                    against the right-hand side as for a warm start).  Needs
 *                    the fused passes down to that level; ignored otherwise,
 *                    and with "warm_start" or "krylov" (default 0)
 *   "merge"          1 = a cycle after which no convergence check follows ends in
 *                    one finest-level pass that does its up pass and the next
 *                    cycle's down pass (prolongation, nu2 + nu1 sweeps, residual,
 *                    restriction) with the node arithmetic of the two passes, so
 *                    iterates and answers are bitwise those of separate passes;
 *                    such a cycle's residual norm is not formed (NaN in the
 *                    history).  Applies with the fused passes on the finest level,
 *                    nu1 + nu2 from 4 to 6, at most 512 radial nodes and one
 *                    plane group; captured graphs ("graph") merge the same
 *                    passes (default 1)
 *   "merge_prefetch" rows the merged pass loads ahead of the one it consumes (1 .. 2; default 1)
 *   "direct"         exact solve of a coarse level (Sec. 3.3 solves the coarsest one
 *                    directly): the V-cycle stops at that level and solves it on every
 *                    plane with the axial generalised eigenvectors of the level's
 *                    separable operator (formed when the plan is built), one radial
 *                    tridiagonal solve per eigenvector, and the inverse transform.
 *                    1 = the first level from 1 on, at or above the bottom kernel's
 *                    first level, with at most 128 interior nodes each way; a level
 *                    above 64 nodes in either direction runs two kernels with FP64
 *                    matrix-core transforms and two workgroups per plane, using the
 *                    level's residual array as scratch.  2 = the first such level with
 *                    at most 64 each way, one workgroup per plane with everything in
 *                    LDS.  0 = off: the V-cycle goes down to the bottom kernel.  Used
 *                    by every FP64 V-cycle, the full-multigrid start included; the
 *                    FP32 inner cycles of "precision" 32 keep the bottom kernel.
 *                    Ignored where no level qualifies (0 .. 2; default 1)
 *   "graph"          1 = the cycles from one convergence check to the next are
 *                    captured once into a HIP graph and replayed (single plane
 *                    group, "timing" 0; default 0).  Setting any option releases
 *                    the captured graphs
 *   "tune_omega"     1 = cylpoisson_autotune also chooses "omega" (point smoother,
 *                    no "krylov"): stretched meshes want more over-relaxation than
 *                    the uniform grids the default is set for (0 .. 1; default 0)
 * Returns CYLPOISSON_OK, CYLPOISSON_EINVAL or CYLPOISSON_ENOMEM. */
int cylpoisson_plan_set_option(cylpoisson_plan* plan, const char* key, double value);

/* Read back an option (keys as for cylpoisson_plan_set_option).  Returns OK or
 * EINVAL (unknown key, NULL argument). */
int cylpoisson_plan_get_option(const cylpoisson_plan* plan, const char* key, double* value);

/* Autotuner for the launch shapes of the fused passes: times short solves (two
 * V-cycles, synthetic charge in two temporary node arrays it allocates and
 * frees) on `stream`, varying one option at a time over candidate values of
 * "chunk_rows", "chunk_rows_coarse", "prefetch" and "groups", and keeps a value
 * only when it is at least 3% faster.  Leaves those four options at the chosen
 * values (read them with cylpoisson_plan_get_option) and every other option as
 * it was.  Results of later solves do not depend on the choice beyond rounding
 * order (tile shapes do not change the arithmetic of a node).  With option
 * "tune_omega" 1 it then measures, for "omega" in 1.0 .. 1.5, the contraction
 * per V-cycle from cycle 2 to cycle 6 of a solve from zero on the same charge,
 * and sets the omega with the smallest contraction if that is under 0.9 times
 * the current omega's (this one changes the iterates).  Blocks; returns OK,
 * ENOMEM or an error of the trial solves. */
int cylpoisson_autotune(cylpoisson_plan* plan, void* stream);

/* Solve `count` independent problems (distinct plans, each with its own grid)
 * together: problem i solves plans[i] with rho[i] -> phi[i] exactly as
 * cylpoisson_solve would, all problems running concurrently on streams of
 * their own (ordered after the work already on `stream`; `stream` waits for
 * all of them on return), so small problems fill the GPU together.  The same
 * tol for all; statuses (optional, count entries) receives each problem's
 * status, and each plan's stats hold its own history.  Returns the first
 * negative status, else NOT_CONVERGED if any problem did not converge, else
 * OK.  Blocks until every problem's result is decided. */
int cylpoisson_solve_batch(cylpoisson_plan* const* plans, const double* const* rho,
                           double* const* phi, int count, double tol, void* stream,
                           int* statuses);

/* Solve for phi given rho (both device node arrays).  Zero initial guess
 * (or phi itself with the option "warm_start"; a guess already within tol
 * returns after 0 cycles), V-cycles until the relative residual
 * (cylpoisson_stats, always relative to the right-hand side) is <= tol or
 * max_cycles is reached (with "precision" = 32: refinement steps of
 * "inner_cycles" FP32 V-cycles each, while the total stays within max_cycles;
 * the residual is always the FP64 one).  rho is read only at interior nodes; every node of
 * phi is written, boundary nodes with the Dirichlet values.  tol > 0.
 * Returns OK, NOT_CONVERGED (phi holds the last iterate), ENONFINITE (phi not
 * written), EINVAL, EDEVICE or EHIP.  Blocks until the result is decided;
 * phi is complete once the stream reaches the end of the enqueued work. */
int cylpoisson_solve(cylpoisson_plan* plan, const double* rho, double* phi, double tol,
                     void* stream);

/* The solve of cylpoisson_solve for callers that cannot allocate device
 * memory (serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * statuses and results as cylpoisson_solve (bit for bit), but the work arrays
 * of the V-cycles -- every level's iterates, right-hand side and residual, the
 * residual-norm partials -- live in a static device array of the library
 * (64 MiB per device, held from the first use of the library on a device
 * until the process ends) instead of the plan's workspace.  The call
 * allocates nothing and creates no stream, event or graph: the options
 * "timing", "groups" and "graph" are ignored for it.  It needs "precision" 64
 * and "krylov" 0, and a plan whose work arrays fit in 64 MiB (about 1.4
 * million unknowns, e.g. 129 x 64 x 129); otherwise EINVAL before any device
 * work.  All calls on one device share its array and each first clears the
 * part it uses (with a kernel on `stream`): calls that overlap on one device
 * race, so issue them on one stream or one after another. */
int cylpoisson_solve_static(cylpoisson_plan* plan, const double* rho, double* phi, double tol,
                            void* stream);

/* Statistics of the last solve (or plane solve).  Returns OK or EINVAL. */
int cylpoisson_get_stats(const cylpoisson_plan* plan, cylpoisson_stats* out);

/* Plan geometry and hierarchy.  Returns OK or EINVAL. */
int cylpoisson_get_info(const cylpoisson_plan* plan, cylpoisson_info* out);

/* Apply the discrete 3-D operator through the mode path:
 *     rho_out = (A_full phi) / s_q   at interior nodes,  0 at boundary nodes,
 * where A_full is the seven-point cell balance of App. A plus the azimuthal
 * three-point term (the left-hand side of Eq. full_finite_volume_row with the
 * boundary nodes of phi as neighbours) and s_q = r_i dr_i dz_k / eps0 with the
 * control-volume widths dr_i, dz_k.  So solving with rho_out returns phi.  Computed as DFT, per-plane
 * A_0 + lambda_m M (Eq. shifted_operator_family), inverse DFT.  Enqueues on
 * stream without synchronising.  Returns OK, EINVAL, EDEVICE or EHIP. */
int cylpoisson_apply(cylpoisson_plan* plan, const double* phi, double* rho_out, void* stream);

/* Forward azimuthal DFT of a node array into planes (convention above).
 * Enqueues without synchronising.  x and planes must not overlap. */
int cylpoisson_dft_forward(cylpoisson_plan* plan, const double* x, double* planes, void* stream);

/* Inverse of cylpoisson_dft_forward: x_j = sum_m x^_m exp(2 pi i m j / N)
 * over all N modes, using conjugate symmetry.  planes and x must not overlap. */
int cylpoisson_dft_inverse(cylpoisson_plan* plan, const double* planes, double* x, void* stream);

/* Solve the per-plane 2-D systems (A_0 + lambda_p M) u_p = b_p of
 * Eq. shifted_operator_family directly, without the DFTs.  b holds the
 * finite-volume right-hand side of every plane at interior nodes (ring
 * entries ignored).  On entry the boundary ring of each plane of u holds
 * that plane's Dirichlet data (interior entries ignored; zero initial
 * guess); on exit the interior holds the solution and the ring is unchanged.
 * Same convergence rule and return values as cylpoisson_solve. */
int cylpoisson_solve_planes(cylpoisson_plan* plan, const double* b, double* u, double tol,
                            void* stream);

/* ---- Learned preconditioner (a network of the brief, not of the paper) ----
 * A three-layer 3x3 convolution network, 4 -> 16 -> 16 -> 2 channels, ReLU
 * after the first two layers, no biases, BF16 operands with FP32 accumulation
 * on the matrix cores, FP32 master weights trained with Adam.  Inputs per
 * interior node of a cos/sin plane pair: the pair's values / the pair's RMS s,
 * (r - r_in)/(r_out - r_in), and lambda mu / D (D the node's diagonal);
 * outputs y give the pair's correction s y / D.  Images for the network are
 * FP32 device arrays [B][H][W][C] (C fastest), zero outside the image.
 * Weights: layers in order, each [9][Cin][Cout], tap = (dy + 1) * 3 + (dx + 1),
 * y[i][j][o] = sum_{tap, c} x[i + dy][j + dx][c] w[tap][c][o]. */

/* New network on the current device, He-normal weights from a SplitMix64
 * stream seeded with `seed`.  NULL on failure. */
cylpoisson_nn* cylpoisson_nn_create(unsigned long long seed);
void cylpoisson_nn_destroy(cylpoisson_nn* nn); /* NULL-safe */
/* Number of weights (all layers). */
int cylpoisson_nn_weight_count(void);
/* Copy the FP32 master weights out / in (host buffers of count floats). */
int cylpoisson_nn_get_weights(const cylpoisson_nn* nn, float* out, int count);
int cylpoisson_nn_set_weights(cylpoisson_nn* nn, const float* in, int count);
/* Gradients of the last cylpoisson_nn_loss_grad (host buffer of count floats). */
int cylpoisson_nn_get_grads(const cylpoisson_nn* nn, float* out, int count);
/* y (B x H x W x 2) = network(x (B x H x W x 4)), device arrays. */
int cylpoisson_nn_forward(cylpoisson_nn* nn, const float* x, float* y, int B, int H, int W, void* stream);
/* Forward, loss = sum over inner pixels (3 from every edge) and both channels of
 * (y - t)^2 / (2 n), and back-propagated weight gradients.  *loss (optional,
 * host) is written after the stream synchronises. */
int cylpoisson_nn_loss_grad(cylpoisson_nn* nn, const float* x, const float* t, int B, int H, int W,
                            double* loss, void* stream);
/* One Adam step (beta 0.9, 0.999, eps 1e-8) with learning rate lr. */
int cylpoisson_nn_adam_step(cylpoisson_nn* nn, float lr, void* stream);
/* Training data from the plain solver: runs `cycles` V-cycles on rho from
 * zero; for the residual r of each iterate it takes the correction c that four
 * red-black SOR sweeps of the solver's smoother compute on A c = r from c = 0,
 * and stores `patches_per_cycle` random 32 x 32 patches (seeded positions over
 * the mode pairs) of r (input) and c (target), appended to the network's
 * store.  The network thus learns a local map the size of its receptive field;
 * the Krylov iteration around it supplies the global coupling.  rho is a
 * device node array of the plan's grid. */
int cylpoisson_nn_collect(cylpoisson_plan* plan, cylpoisson_nn* nn, const double* rho, int cycles,
                          int patches_per_cycle, unsigned long long seed, void* stream);
long long cylpoisson_nn_patch_count(const cylpoisson_nn* nn);
/* Adam over the stored patches in batches, `epochs` passes; *loss_out = the
 * last epoch's mean loss. */
int cylpoisson_nn_train(cylpoisson_nn* nn, int epochs, int batch, float lr, double* loss_out, void* stream);
/* Attach (or with NULL detach) the network used by the option "krylov"; the
 * plan does not own it. */
int cylpoisson_plan_set_net(cylpoisson_plan* plan, cylpoisson_nn* nn);

/* Thread-local message describing the last failure in this thread ("" if none). */
const char* cylpoisson_last_error(void);

/* Status of the last cylpoisson_plan_create or cylpoisson_plan_create_mesh in
 * this thread: OK after a plan was returned; after NULL, EINVAL (arguments or
 * geometry rejected), ENOMEM (a host or device allocation failed, e.g. a
 * workspace larger than the device memory) or EHIP (another HIP failure).
 * Every allocation of a failed creation is released. */
int cylpoisson_last_status(void);

/* Static description of a status code. */
const char* cylpoisson_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* CYLPOISSON_H */
