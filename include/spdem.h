/*
 * spdem: superparameterised sea-ice floe DEM on one MI355X (gfx950).
 *
 * Method: Deng, Stechmann & Chen, "Particle-continuum multiscale modeling of
 * sea ice floes".  Every coarse grid cell runs its own doubly periodic DEM of
 * rigid disk floes (Sec. 3.1); one fine step integrates the DEM system of
 * Sec. 2.1 (ocean drag and drag torque, Hooke normal and Coulomb-capped
 * tangential contact forces and their spin torques); the per-cell statistics
 * of the floes (Sec. 2.3, Sec. 3.2) drive one Lax-Friedrichs step of the
 * moment equations for mass density, momentum and spin angular momentum, with
 * the Oseen treatment of the momentum advection (Sec. 3.2).
 *
 * Conventions shared by every call:
 *   - cells are numbered c = iy * nx + ix; floes are stored sorted by cell;
 *   - positions are cell-local, as unsigned 32-bit fractions of the cell side:
 *     x = cell_lx * xi / 2^32 (periodic wrap is the natural 2^32 wrap);
 *   - velocities u, v (m/s), spin omega (1/s), angle theta (rad), radius r (m)
 *     and thickness h (m) are float32; mass m = rho_ice h pi r^2, I = m r^2;
 *   - the ocean current is prescribed (Sec. 2.1):
 *     u_o(X, Y) = (u0, v0) + sum_m (au_m, av_m) sin(kx_m X + ky_m Y + phase_m)
 *     at global X = (ix + xi / 2^32) cell_lx, with curl dv_o/dX - du_o/dY;
 *   - all calls are asynchronous on the context's stream except those marked
 *     "synchronises"; no call throws; errors are returned as sp_status and the
 *     message of the last failure is kept per context (sp_last_error);
 *   - faults detected on the device (coincident centres, non-finite state,
 *     CFL > 1, contact-list overflow) are latched in a device flag and
 *     returned by the next synchronising call;
 *   - a context is thread-compatible, not thread-safe.
 */
#ifndef SPDEM_H
#define SPDEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sp_ctx sp_ctx;

typedef enum {
    SP_OK = 0,
    SP_EINVAL = -1,     /* bad argument: size, range, null pointer, r_max >= L/4 */
    SP_ENOMEM = -2,     /* device allocation failed */
    SP_EDEVICE = -3,    /* HIP runtime error */
    SP_ECFL = -4,       /* continuum CFL number exceeded 1 (Sec. 3.2) */
    SP_EOVERLAP = -5,   /* two floe centres coincide: contact normal undefined */
    SP_ENAN = -6,       /* non-finite floe state */
    SP_ESTATE = -7,     /* call out of order (e.g. step before set_floes) */
    SP_ECAPACITY = -8,  /* a cell exceeds the per-cell floe or contact capacity */
    SP_EWALL = -9       /* a floe crossed a wall (SP_WALL_X) */
} sp_status;

/* sp_params.flags */
#define SP_OCEAN_OFF 1u       /* no drag, no drag torque */
#define SP_FORWARD_EULER 2u   /* positions advance with the old velocities */
#define SP_NO_CONTINUUM 4u    /* skip the coarse Lax-Friedrichs update */
/* Tangential contact force as the incremental spring of the Cundall-Strack
 * model the paper cites for it (Sec. 2.1) instead of the printed viscous law:
 * each contact keeps its tangential displacement xi (zero when the contact
 * begins, forgotten when it ends), xi grows by v_t dt per step, the force is
 * c G xi t with G read as a shear modulus (N/m^2), and where |c G xi| would
 * pass mu |f_n| the contact slips: the force takes the Coulomb limit and xi
 * the displacement that gives it.  History: SP_SPRING_CAP contacts per floe
 * (SP_ECAPACITY beyond), kept in device memory and, in blocked launches
 * (sp_set_step_block, the coupled cadence of sp_set_coupling), staged in LDS
 * for the block (80 B per floe more per cell): the same floe state bit for
 * bit as one launch per step.  The plain step falls back to one launch per
 * step when some cell's blocked launch would not fit the 160 KB of LDS; the
 * coupled cadence returns SP_ECAPACITY there.  Not with the hybrid, closure
 * sampling or the autotuner (SP_ESTATE). */
#define SP_TANGENTIAL_SPRING 8u
#define SP_SPRING_CAP 8
/* Walls at x = 0 and at the far x edge, the boundary of the paper's
 * scenario of floes driven into a fixed wall (Sec. 4.4); periodic in y.
 * sp_ctx (sp_params.flags): the coarse model takes a zero (Dirichlet)
 * boundary condition on the floe concentration in x: beyond the first and
 * the last column of cells lies a ghost cell with zero state (rho, P_x, P_y,
 * P_w) and zero coefficients <v> in every Lax-Friedrichs step, on every path
 * (plain, blocked, coupled); the cell DEMs stay doubly periodic (Sec. 3.1).
 * Not with the hybrid or closure sampling (SP_ESTATE).
 * sp_gdem (sp_gdem_params.flags): the global DEM is periodic in y only, and a
 * floe whose centre lies within its radius of a wall is in contact with it:
 * the contact law of Sec. 2.1 with the wall as a fixed body, overlap
 * delta = d - r (d the centre's distance to the wall), chord
 * c = 2 sqrt(r^2 - d^2), normal force c E delta towards the floe, tangential
 * force c G v_t capped at mu |f_n| with v_t the floe's contact-point velocity
 * along the wall, spin torque r f_t; each wall contact counts as a contact.
 * A floe whose centre passes a wall latches SP_EWALL. */
#define SP_WALL_X 16u

/* sp_params.schedule: how a cell's contact candidates are enumerated.
 * Every schedule yields the same contact set and, because each floe sums its
 * contacts in ascending partner index, the same floe state bit for bit. */
#define SP_SCHED_AUTO 0       /* binned where the cell allows >= 3 bins per side */
#define SP_SCHED_ALLPAIRS 1   /* every floe against every floe of its cell */
#define SP_SCHED_BINNED 2     /* square sub-bins of side >= 2 r_max, 3x3 sweep */

/* sp_read_moments(which) */
#define SP_MOMENTS_DEM 0        /* [ncells][SP_NMOM] statistics of the current floe state */
#define SP_MOMENTS_CONTINUUM 1  /* [ncells][4] continuum state Q = (rho, P_x, P_y, P_w) */

/* DEM statistics per cell, in this order (FP64 sums over the cell's floes):
 * n, M = sum m, P_x = sum m u, P_y = sum m v, L = sum I omega, U_x = sum u,
 * U_y = sum v, S_vx, S_vy = sum of ocean drag forces, S_w = sum of drag
 * torques, A_ice = sum pi r^2.  The continuum coefficients are U/n and the
 * sources S/A (A = cell area); Q^0 = (M, P_x, P_y, L) / A of the initial state
 * (Algorithm 1 initialises the coarse model from DEM data). */
#define SP_NMOM 11

#define SP_MAX_MODES 16        /* ocean Fourier modes */
#define SP_MAX_CELL_FLOES 1024 /* floes per cell (LDS-resident cell) */
#define SP_CONTACT_CAP 24      /* contact candidates per floe: contacts and the
                                  neighbours within the candidate-list skin */

typedef struct {
    int32_t nx, ny;           /* coarse grid = one DEM per cell (Sec. 3.1) */
    double cell_lx, cell_ly;  /* cell size (m); also the coarse spacing dX, dY */
    double rho_ice;           /* ice density (kg/m^3) */
    double rho_ocean;         /* ocean density (kg/m^3) */
    double cd;                /* ocean drag coefficient d_o */
    double E;                 /* normal stiffness per unit chord length (N/m^2) */
    double G;                 /* tangential viscous coefficient per unit chord (N s/m^2);
                                 with SP_TANGENTIAL_SPRING the shear modulus (N/m^2) */
    double mu;                /* Coulomb friction coefficient */
    uint32_t flags;           /* SP_OCEAN_OFF | SP_FORWARD_EULER | SP_NO_CONTINUUM |
                                 SP_TANGENTIAL_SPRING | SP_WALL_X */
    int32_t schedule;         /* SP_SCHED_* */
} sp_params;

/* Create a context on the current HIP device: the coarse grid of one DEM per
 * cell and the constants of the floe system (Algorithm 1, initialisation of
 * the time-marching parameters; Sec. 2.1 constants; Sec. 3.1 one periodic DEM
 * per coarse cell).  `stream` is a hipStream_t the caller owns (e.g.
 * torch.cuda.current_stream().cuda_stream) or NULL, in which case the context
 * creates its own default-priority stream.
 * Errors: SP_EINVAL (null out, nx/ny < 1, non-positive sizes or constants),
 * SP_EDEVICE. */
sp_status sp_create(const sp_params* params, void* stream, sp_ctx** out);

/* Release every device buffer the context owns.  NULL is ignored. */
void sp_destroy(sp_ctx* ctx);

/* Message of the last failing call on this context (never NULL). */
const char* sp_last_error(const sp_ctx* ctx);

/* Prescribed ocean current (Sec. 2.1).  Host arrays of nmodes doubles, copied.
 * 0 <= nmodes <= SP_MAX_MODES.  May be called before or after sp_set_floes.
 * Errors: SP_EINVAL. */
sp_status sp_set_ocean(sp_ctx* ctx, double u0, double v0, int32_t nmodes, const double* kx,
                       const double* ky, const double* au, const double* av, const double* phase);

/* Floe state from host arrays (copied): Algorithm 1's initialisation of the N
 * floes, each with the position, velocity, spin, angle, radius and thickness
 * of Sec. 2.1, assigned to the coarse cell that holds it (Sec. 3.1).
 * counts[ncells] floes per cell,
 * sum(counts) = n; per-floe arrays of length n sorted by cell.  omega and theta
 * may be NULL (zero).  Resets the continuum to the statistics of this state.
 * Errors: SP_EINVAL (sizes, r <= 0, h <= 0, r_max >= min(cell_lx, cell_ly)/4),
 * SP_ECAPACITY (a cell above SP_MAX_CELL_FLOES), SP_ENOMEM, SP_EDEVICE. */
sp_status sp_set_floes(sp_ctx* ctx, int64_t n, const int32_t* counts, const uint32_t* xi,
                       const uint32_t* yi, const float* u, const float* v, const float* omega,
                       const float* theta, const float* r, const float* h);

/* The same from device buffers (e.g. torch tensors), copied on the stream;
 * counts stays a host array.  Synchronises (radius validation). */
sp_status sp_set_floes_device(sp_ctx* ctx, int64_t n, const int32_t* counts, const void* xi,
                              const void* yi, const void* u, const void* v, const void* omega,
                              const void* theta, const void* r, const void* h);

/* Advance nsteps fine steps of size dt (s): each step is one DEM step of every
 * cell fused with the statistics of the pre-step state, then (unless
 * SP_NO_CONTINUUM) one Lax-Friedrichs step of the continuum driven by those
 * statistics (coarse step = fine step, N0 = N1 = 1 in Algorithm 1).  With a
 * cadence N0 > 1 set by sp_set_coupling, the steps follow that cadence instead.
 * Asynchronous.  Errors: SP_EINVAL (dt <= 0, nsteps < 0), SP_ESTATE. */
sp_status sp_step(sp_ctx* ctx, double dt, int64_t nsteps);

/* Two-way coupling cadence of sp_step (Algorithm 1: coupling loop; Sec. 3.2
 * coarse step; Sec. 3.3 gradual coarse-to-fine update).  The next sp_step call
 * starts a new run of the algorithm at fine step j = 1 from the current floes
 * and coarse state.  Fine step j advances every cell DEM and keeps the
 * statistics of its pre-step state; at j = k N0 the coarse model advances by
 * dT = N0 dt in N1 Lax-Friedrichs sub-steps of dT / N1, driven by the mean of
 * the window's N0 statistics, and the DEM cell values X0 = (M, P_x, P_y, L) / A
 * of the state reached are kept; from the second coarse step on, at fine steps
 * whose r = j mod N0 is a nonzero multiple of n_t, every cell with floes is
 * re-synchronised (radii scaled by one factor, then uniform velocity and spin
 * shifts, as sp_resync_cells) to X0 + (r / N0) (Q - X0), Q the latest coarse
 * state.  At each coarse step the contact search (sub-bins, skin) is
 * re-planned, when needed, for the largest radius the next coarse step's
 * updates can produce (a cell's radii scale by sqrt(rho_target / rho_X0) and
 * its targets lie between X0 and Q), so no update is limited by it; only a
 * cell whose radii would pass a quarter of the cell (the limit of the periodic
 * cell DEM) is scaled up to that ("clamped"), and a target with rho <= 0
 * leaves its cell unchanged ("invalid").  Each coarse step synchronises the
 * stream once (a 4-byte read of that radius).  dt is the dt of each sp_step
 * call; a coarse step uses N0 times the dt of the call that completes it.
 * N0 = N1 = n_t = 1 is the plain step.  Between coarse steps
 * SP_MOMENTS_CONTINUUM reads the latest coarse state.  With a step block
 * k > 1 (sp_set_step_block) the fine steps up to each update run as blocked
 * launches of at most k steps,
 * the update done inside the launch that ends at it.  Cadence state lives in
 * the context: a ring of N0 x ncells x 128 B statistics.
 * Errors: SP_EINVAL (a value < 1, N0 or N1 > SP_MAX_COUPLING), SP_ESTATE
 * (N0 > 1 with SP_NO_CONTINUUM or an active hybrid), SP_ENOMEM at the first
 * coupled sp_step.  sp_hybrid_set, sp_step_hybrid, sp_closure_sample and
 * sp_profile_steps return SP_ESTATE while N0 > 1. */
#define SP_MAX_COUPLING 65536
sp_status sp_set_coupling(sp_ctx* ctx, int32_t N0, int32_t N1, int32_t n_t);

/* The cadence, then counted since the last sp_set_coupling (or sp_set_floes):
 * coarse-to-fine update passes, contact-search re-plans, clamped and invalid
 * cell updates.  Any pointer may be NULL.  Synchronises. */
sp_status sp_get_coupling(sp_ctx* ctx, int32_t* N0, int32_t* N1, int32_t* n_t, int64_t* nudges,
                          int64_t* replans, int64_t* clamped, int64_t* invalid);

/* Save and restore a simulation (Algorithm 1 ends by saving the data of the
 * run).  sp_save writes to the file at `path` everything a later sp_step reads:
 * the floe state (all eight per-floe arrays, counts per cell), the continuum
 * state of the current level, the step counters, the candidate lists and
 * their displacement bounds, the contact and candidate counters, the largest
 * CFL number, the ocean, every cell's reduced DEM and, with
 * SP_TANGENTIAL_SPRING, the contact history; a continuum update still
 * pending from the last step is saved as pending, with its operands.  It
 * waits for the stream and does not change the simulation.  sp_load reads such a file into a
 * context created with the same sp_params (grid, constants, flags, schedule):
 * it sets the ocean and the floes as sp_set_ocean and sp_set_floes do (which
 * removes a hybrid and restarts the coupling cadence), then restores the rest,
 * so that the steps that follow give the same floe state and continuum bit for
 * bit as the saved context would have.  The loading context keeps its own
 * batching, step block and cadence settings.  Host byte order; the file is
 * not portable across library versions.  Both synchronise.
 * Errors: SP_EINVAL (null path, unreadable, truncated or foreign file, other
 * parameters), SP_ESTATE (sp_save before sp_set_floes, with an active hybrid,
 * or with N0 > 1), SP_EDEVICE (a write failed), the errors of sp_set_floes,
 * and a latched device fault (sp_save). */
sp_status sp_save(sp_ctx* ctx, const char* path);
sp_status sp_load(sp_ctx* ctx, const char* path);
/* Number of floes of the current state and of cells (either may be NULL). */
sp_status sp_get_size(sp_ctx* ctx, int64_t* nfloes, int32_t* ncells);

/* Block until the stream is idle; returns the first latched device fault. */
sp_status sp_synchronize(sp_ctx* ctx);

/* The cell averages the coarse model consumes (eq. meang and Sec. 2.3 for the
 * DEM statistics; Sec. 3.2 for the coarse state rho, rho v, P_w).
 * Copy moments to a caller-owned host array: [ncells][SP_NMOM] for
 * SP_MOMENTS_DEM (statistics of the current state, drag at the current
 * state) or [ncells][4] for SP_MOMENTS_CONTINUUM.  Synchronises. */
sp_status sp_read_moments(sp_ctx* ctx, int32_t which, double* out);

/* For callers that cannot allocate device memory (serving loops and harnesses
 * that forbid hipMalloc): sp_read_moments without any allocation.  The same
 * values as sp_read_moments bit for bit, into the same caller-owned host
 * array out ([ncells][SP_NMOM] or [ncells][4]); the rows are staged in a
 * static device array of the library (8 MiB per device, held until the
 * process ends) instead of buffers it allocates, so it serves contexts of at
 * most 65,536 cells.  Every call on a device uses that device's one array:
 * calls that overlap on one device (from several threads) race; each call
 * writes every row it reads, so nothing carries over between calls.
 * Synchronises.  Errors: those of sp_read_moments, SP_ECAPACITY (more than
 * 65,536 cells), SP_EDEVICE (the array's address could not be taken). */
sp_status sp_read_moments_noalloc(sp_ctx* ctx, int32_t which, double* out);

/* The fine-scale state of Sec. 2.1 (positions, velocities, spins, angles,
 * radii of every floe, in the cell-sorted order of sp_set_floes).
 * Copy the floe state to caller-owned host arrays of length n (any may be NULL).
 * Synchronises. */
sp_status sp_read_floes(sp_ctx* ctx, uint32_t* xi, uint32_t* yi, float* u, float* v,
                        float* omega, float* theta, float* r);

/* Contact pairs of the current state as global floe indices l < j, sorted by
 * (l, j); writes min(count, cap) pairs and sets *count.  Debug/test call: the
 * decision is the one the step kernels take.  Synchronises. */
sp_status sp_read_pairs(sp_ctx* ctx, int64_t cap, int32_t* l, int32_t* j, int64_t* count);

/* Counters since the last sp_set_floes: contacts summed over steps and floe
 * pairs (each pair counted once), steps taken, and the largest continuum CFL
 * number seen.  Synchronises. */
sp_status sp_get_stats(sp_ctx* ctx, int64_t* contacts, int64_t* steps, double* max_cfl);

/* Run nsteps steps like sp_step but launched one by one (no graph replay),
 * with one pair of HIP events recorded on the context's stream before the
 * first and after the last step's launches, and return the mean duration of a
 * step's DEM launches (ms) in *dem_ms: the elapsed time over nsteps, which
 * holds the kernels and the short gaps between back-to-back launches; *lf_ms
 * is 0 because the continuum update runs inside those launches.  With blocked
 * steps (sp_set_step_block) whole blocks run (nsteps rounded up to a multiple
 * of k), events bracket every block's DEM launches, *dem_ms is their time per
 * step and *lf_ms the time of the continuum updates per step.  The state
 * advances exactly as with sp_step.  Synchronises. */
sp_status sp_profile_steps(sp_ctx* ctx, double dt, int64_t nsteps, double* dem_ms, double* lf_ms);

/* Batching of cells with uneven floe counts.  Cells with floes are grouped by
 * count into SP_NUM_BUCKETS buckets (<= 64, <= 128, <= 256, <= 512, <= 1024
 * floes; cells without floes take only the continuum update); each
 * bucket is one launch per step over its cells, costliest first, with W
 * wavefronts per cell (W = 1, 2, 4 or 8: one wavefront per small cell up to a
 * tile of 8 wavefronts per large cell) and either one workgroup per cell group
 * or persistent workgroups: as many as are resident at once, each striding
 * over the cells and loading the next cell's floes while it processes one.
 * Every choice gives the same
 * floe state bit for bit; cell statistics agree to FP64 rounding (the
 * reduction tree follows W).
 * sp_get_batching: cells[b], waves[b], persistent[b] for each bucket (any may be NULL).
 * sp_set_batching: choose waves[b] and persistent[b] (0/1) for every bucket.
 * Errors: SP_EINVAL. */
#define SP_NUM_BUCKETS 5
sp_status sp_get_batching(sp_ctx* ctx, int32_t* cells, int32_t* waves, int32_t* persistent);
sp_status sp_set_batching(sp_ctx* ctx, const int32_t* waves, const int32_t* persistent);

/* Tune the batching of the launches sp_step runs, on a scratch copy of the
 * floe state (the simulation is not advanced; candidate lists are rebuilt at
 * the next step).  With blocked steps (block length > 1 at the plain cadence,
 * see sp_set_step_block): every non-empty bucket alone over the wavefronts per
 * cell of its blocked launches that hold one floe per lane (W = 1, 2, 4, 8,
 * 16), then the block length (16, 32 or 64 steps) over the whole step; each
 * variant one warm-up launch and the minimum of reps timed launches; *best_ms
 * receives the best whole step's time per step.  Otherwise (per-step launches)
 * every (waves, persistent) variant of every bucket's per-step kernel, reps
 * repetitions of two steps each; *best_ms the summed best step time of the
 * buckets.  *best_ms may be NULL.  Synchronises.
 * Errors: SP_EINVAL, SP_ESTATE, SP_ENOMEM, SP_EDEVICE. */
sp_status sp_autotune(sp_ctx* ctx, double dt, int32_t reps, double* best_ms);
/* Wavefronts per cell of each bucket's blocked launches (0 for an empty
 * bucket), as sp_autotune or the defaults set them. */
sp_status sp_get_block_waves(sp_ctx* ctx, int32_t* waves);

/* Temporal blocking of the plain step (coarse step = fine step): with k > 1,
 * sp_step runs whole blocks of k steps as one DEM launch per count bucket in
 * which every cell keeps its floes and candidate lists in LDS for the k steps
 * (the cell DEMs never read the continuum at this cadence), each step's
 * statistics going to a k-slot ring, followed by the k continuum updates;
 * a call's remaining steps (fewer than k) run as one block of their own
 * length, so every step of sp_step is blocked and none captures a graph.  Blocked launches hold one floe per lane: a
 * bucket whose cells exceed 64 W floes runs them with W = 8 (up to 512 floes)
 * or 16 (up to SP_MAX_CELL_FLOES).  Applies to sp_step with N0 = 1 (the coupled cadence
 * blocks its stretches between
 * coarse-to-fine updates, the hybrid its DEM cells between checks: see
 * sp_set_coupling and sp_step_hybrid).  The floe state is the same
 * bit for bit as with k = 1; statistics are summed in another fixed order.
 * With SP_TANGENTIAL_SPRING the contact history is staged in LDS as well.
 * Ring: k x ncells x 128 B.  Default 32.  Errors: SP_EINVAL (k outside
 * [1, SP_MAX_STEP_BLOCK]). */
#define SP_MAX_STEP_BLOCK 1024
sp_status sp_set_step_block(sp_ctx* ctx, int32_t k);
/* The block length and whether blocked steps currently apply (1) or not (0). */
sp_status sp_get_step_block(sp_ctx* ctx, int32_t* k, int32_t* active);
/* Work counted by blocked steps since sp_set_floes: candidate-list entries
 * tested (over floes and steps) and the steps taken in blocks (either may be
 * NULL).  Synchronises. */
sp_status sp_get_work(sp_ctx* ctx, int64_t* candidate_tests, int64_t* blocked_steps);

/* sp_step replays runs of `chunk` steps as one captured HIP graph (default 16;
 * 0 disables capture; must be even).  Results are identical either way. */
sp_status sp_set_graph_chunk(sp_ctx* ctx, int32_t chunk);

/* ------------------------------------------------------------------------
 * Learned closure.  The paper closes the momentum equation's stress term
 * only through the fine-scale DEM (Sec. 2.3); this network maps a cell's
 * coarse neighbourhood to its moment tendencies so that cells away from the
 * marginal ice zone can skip the DEM.  Architecture: 45 -> 128 -> 128 -> 128
 * -> 4, GELU (erf form), bfloat16 weights and activations, FP32 accumulation
 * on MFMA, FP32 master weights, Adam (beta = 0.9, 0.999, eps = 1e-8), mean
 * squared error on normalised targets.  Parameters are one flat FP32 vector of
 * SP_MLP_NPARAMS entries: W1 [128 x 45], b1, W2 [128 x 128], b2, W3, b3,
 * W4 [4 x 128], b4 (row-major, W[o][i] multiplies input i into output o).
 * Inputs per cell (SP_MLP_IN): a continuum state (rho, P_x, P_y, P_w) on the
 * 3 x 3 neighbourhood row by row from the south-west (36), the ocean current
 * and curl at the cell centre (3), the cell's A_ice / A, mean h and
 * r2m = sum m r^2 / sum m (3), and the relative velocity and spin of its
 * reduced DEM (below) at the current time (3).  Outputs (SP_MLP_OUT): moment
 * tendencies d(rho, P_x, P_y, P_w)/dt.  Inputs and outputs are normalised
 * per column by the stored means and standard deviations.
 *
 * Reduced DEM of a cell: its floes seen as one body under the drag laws of
 * Sec. 2.1.  Taken from the floes at time t0 (mean velocity U = sum v / n,
 * mean spin W = L / (M r2m)), its velocity and spin relative to the ocean
 * current u_o and half-curl at the cell centre relax in the closed form of a
 * single floe's quadratic drag, du(t) = du(t0) / (1 + k_v |du(t0)| (t - t0)),
 * dW(t) = dW(t0) / (1 + (k_w / r2m) |dW(t0)| (t - t0)), with the cell's
 * k_v = C_d rho_o sum pi r^2 / sum m and k_w = C_d rho_o sum pi r^5 / sum m.
 * Its statistics are the coefficient <v> = u_o - du and the sources per unit
 * area rho_f k_v |du| du and rho_f k_w |dW| dW, rho_f = sum m / A.  Every
 * cell's reduced DEM is taken from its floes when they are set, when the
 * ocean is set, and when the cell is re-synchronised.
 * All data pointers of the sp_mlp_* calls are device pointers except where
 * marked host.  The object runs on its own stream (or the one given), in
 * stream order: device inputs must be ready on that stream when a call is
 * made, and sp_mlp_forward's output is ready once the stream reaches it
 * (calls that return host values synchronise the stream). */
#define SP_MLP_NPARAMS 39428
#define SP_MLP_IN 45
#define SP_MLP_OUT 4
typedef struct sp_mlp sp_mlp;
sp_status sp_mlp_create(void* stream, sp_mlp** out);
void sp_mlp_destroy(sp_mlp* net);
const char* sp_mlp_last_error(const sp_mlp* net);
/* host params[SP_MLP_NPARAMS]; set also resets the Adam state */
sp_status sp_mlp_set_params(sp_mlp* net, const float* params);
sp_status sp_mlp_get_params(sp_mlp* net, float* params);
/* host arrays: x_mean, x_std [SP_MLP_IN], y_mean, y_std [SP_MLP_OUT]; a zero
 * x_std drops that input */
sp_status sp_mlp_set_norm(sp_mlp* net, const float* x_mean, const float* x_std, const float* y_mean,
                          const float* y_std);
sp_status sp_mlp_get_norm(sp_mlp* net, float* x_mean, float* x_inv_std, float* y_mean, float* y_std);
/* per-column mean and standard deviation of a device data set X [n][45], T [n][4] */
sp_status sp_mlp_fit_norm(sp_mlp* net, const float* X, const float* T, int64_t n);
/* y [M][4] = network(x [M][45]), de-normalised */
sp_status sp_mlp_forward(sp_mlp* net, const float* x, int64_t M, float* y);
/* gradient of the loss over B samples into host grad[SP_MLP_NPARAMS]; *loss (host) */
sp_status sp_mlp_gradient(sp_mlp* net, const float* X, const float* T, int32_t B, float* grad, float* loss);
/* one Adam step on the B rows of X, T listed in rows (device, may be NULL = first B) */
sp_status sp_mlp_train_step(sp_mlp* net, const float* X, const float* T, const int32_t* rows, int32_t B,
                            float lr, float* loss);
/* floor(n / batch) Adam steps over X, T in the order of perm (device [n]); *mean_loss (host) */
sp_status sp_mlp_train_epoch(sp_mlp* net, const float* X, const float* T, const int32_t* perm, int64_t n,
                             int32_t batch, float lr, float* mean_loss);
/* Input noise of the training steps (sp_mlp_train_step, sp_mlp_train_epoch;
 * never sp_mlp_gradient or sp_mlp_forward), the data augmentation of the
 * closure's training: in Adam step s (the number of steps the network took
 * before it) input f < nfeat of row i of X gets sd[f] (host, raw input units)
 * times a standard normal from the counter-based generator SplitMix64 of
 * (seed, s, i, f / 2) through the Box-Muller transform (features f and f + 1
 * of an even f share one pair), so that a run repeats bit for bit.  With noise
 * on, a training call first writes a noisy copy of its rows (all of an
 * epoch's, in the order its steps read them) into a buffer the network owns
 * (grown as needed, 196 B per row).  nfeat = 0 turns it off.
 * Errors: SP_EINVAL (nfeat outside [0, SP_MLP_IN], sd null for nfeat > 0, a
 * negative or non-finite sd); the training calls also SP_ENOMEM. */
sp_status sp_mlp_set_input_noise(sp_mlp* net, int32_t nfeat, const float* sd, uint64_t seed);
/* closure inputs of every cell of the current state Q into x [ncells][45] (device) */
sp_status sp_closure_features(sp_ctx* ctx, float* x);
/* Samples of sp_closure_sample.  SP_TEND_FULL: features of the current state
 * Q, targets (Q_new - Q) / dt.  SP_TEND_RESIDUAL: the part of the update the
 * reduced DEMs do not give, the training target of the hybrid's network:
 * features of the base-updated state Q_b, targets (Q_new - Q_b) / dt, where
 * Q_b is the continuum update of Sec. 3.2 with the statistics of every cell
 * taken from its reduced DEM. */
#define SP_TEND_FULL 0
#define SP_TEND_RESIDUAL 1
/* one training sample per cell: inputs of `mode` into x [ncells][45], one
 * step of size dt, tendencies of `mode` into t [ncells][4] (device).
 * Errors: SP_EINVAL (null buffer, dt <= 0, unknown mode), SP_ESTATE,
 * SP_EDEVICE. */
sp_status sp_closure_sample(sp_ctx* ctx, double dt, int32_t mode, float* x, float* t);

/* ------------------------------------------------------------------------
 * Coarse-to-fine re-synchronisation (Sec. 3.3, the nudging of the fine state
 * towards the coarse one, with all its sub-steps taken at once).
 * Moves the floes of each listed cell to host targets[i] = (rho, P_x, P_y,
 * P_w) per unit area: every radius is multiplied by s = sqrt(rho A / M) (the
 * increment proportional to the radius that gives the cell mass rho A), then
 * every floe of the cell gets the velocity shift (A P - sum m v) / M and the
 * spin shift (A P_w - sum I w) / sum I, with M and I of the rescaled floes
 * (FP64 sums, results stored FP32).  A radius may not exceed the contact
 * search radius fixed when the floes were set (the largest radius then): a
 * cell whose scale would pass it is scaled only up to it, keeps less mass
 * than its target, and is counted in *clamped (host, may be NULL).
 * cells (host, ncl distinct indices) and targets (host, [ncl][4]) are read
 * only during the call.  Errors: SP_EINVAL (index out of range or repeated,
 * rho <= 0 or non-finite target for a cell with floes, nonzero target for
 * an empty cell; nothing is changed then), SP_ESTATE (no floes), SP_ENOMEM,
 * SP_EDEVICE.  The cells' reduced DEMs restart from the re-synchronised
 * floes.  Synchronises. */
sp_status sp_resync_cells(sp_ctx* ctx, int32_t ncl, const int32_t* cells, const double* targets,
                          int32_t* clamped);

/* ------------------------------------------------------------------------
 * DEM + closure hybrid.  closure_cells (host, [ncells], copied) flags the
 * cells whose continuum state advances without their DEM (a flag on a cell
 * without floes is ignored: its plain update needs no DEM work):
 * Q <- Q_b + dt T(features of Q_b), with Q_b and the features of
 * SP_TEND_RESIDUAL and T the output of a network trained on its targets.  All
 * other cells run the DEM step and the continuum update of Sec. 3.2, which
 * takes the reduced DEM's <v> as the coefficient of a neighbouring closure
 * cell.  A closure cell's floes stay frozen, except in the check pool: up to
 * 4 check_cells closure cells spread evenly over them, whose DEMs keep
 * stepping (their statistics unused), so that their floes are the plain
 * method's (the cells' DEMs do not interact).  Every check_every steps the
 * next check_cells pool cells in closure mode (round robin) are checked:
 * their statistics give the plain method's residual tendency T_dem, and a
 * cell whose closure residual T (T = 0 once its reduced DEM is older than
 * net_window) misses it so much that check_every dt |T - T_dem| exceeds tol
 * (|Q_cell| + 0.01 mean |Q| of the sample) in any component runs the DEM for
 * the next fallback_steps steps, after which its reduced DEM restarts from
 * its floes.  Every checked cell's reduced DEM restarts from its floes.  With
 * net_window > 0 the
 * network's term is applied to a closure cell only during the first
 * net_window seconds of its reduced DEM (the relaxation transient the network
 * is trained on); later the reduced DEM alone carries the cell.  A null
 * closure_cells removes the hybrid.  The network must stay alive and
 * unchanged while the hybrid is set; it runs on the simulation's stream.
 * Setting new floes removes the hybrid.
 * Errors: SP_EINVAL, SP_ESTATE (no floes, or SP_NO_CONTINUUM), SP_ENOMEM,
 * SP_EDEVICE.  Synchronises. */
sp_status sp_hybrid_set(sp_ctx* ctx, sp_mlp* net, const uint8_t* closure_cells, int32_t check_every,
                        int32_t check_cells, double tol, int32_t fallback_steps, double net_window);
/* nsteps hybrid steps of size dt (asynchronous except at checks and mode
 * changes).  With a step block k > 1 (sp_set_step_block) the DEM-mode cells'
 * steps up to the next check or the end of a fallback window run as blocked
 * launches of at most k steps, followed by each step's closure and continuum
 * work in order; the floe state is the same bit for bit as with k = 1.
 * Errors: SP_EINVAL, SP_ESTATE (no hybrid), SP_EDEVICE. */
sp_status sp_step_hybrid(sp_ctx* ctx, double dt, int64_t nsteps);
/* current DEM-mode and closure-mode cell counts, checks made, fallbacks
 * triggered (host, any may be NULL).  Errors: SP_ESTATE (no hybrid). */
sp_status sp_hybrid_stats(sp_ctx* ctx, int32_t* dem_cells, int32_t* closure_cells, int64_t* checks,
                          int64_t* fallbacks);

/* Schedule actually used for the current floes (after SP_SCHED_AUTO), and the
 * sub-bins per side it uses (1 for all-pairs). */
sp_status sp_get_schedule(sp_ctx* ctx, int32_t* schedule, int32_t* bins_x, int32_t* bins_y);

/* ------------------------------------------------------------ global DEM
 * The reference of the paper's error study (Sec. 4): one DEM of the same floe
 * system (Sec. 2.1: contact law, ocean drag and torque, semi-implicit update)
 * over the whole doubly periodic domain, floes free to cross coarse cells and
 * every pair a potential contact.  Positions are unsigned 32-bit fractions of
 * the domain: X = lx * xi / 2^32; the ocean is evaluated at X as for sp_ctx.
 * Contacts are searched in sub-bins of side >= 2 r_max (3 x 3 sweep, one
 * sub-bin along an axis with fewer than 3), re-binned before every step by a
 * stable counting sort (the order a stable sort by sub-bin of the current
 * order gives; one launch, the counts made by the previous step's launch);
 * decisions and forces match the cell DEM's.  Statistics for any coarse grid
 * are read with sp_gdem_coarse_moments. */
typedef struct sp_gdem sp_gdem;

typedef struct {
    double lx, ly;            /* domain size (length unit of the inputs) */
    double rho_ice, rho_ocean, cd, E, G, mu;   /* as sp_params */
    uint32_t flags;           /* SP_OCEAN_OFF | SP_FORWARD_EULER | SP_WALL_X */
} sp_gdem_params;

/* Create a context on the current device (stream as sp_create).
 * Errors: SP_EINVAL (null, non-positive size or density, negative constant),
 * SP_EDEVICE. */
sp_status sp_gdem_create(const sp_gdem_params* params, void* stream, sp_gdem** out);
/* Release the context; NULL is ignored. */
void sp_gdem_destroy(sp_gdem* g);
/* Message of the last failing call (never NULL). */
const char* sp_gdem_last_error(const sp_gdem* g);
/* Ocean current, as sp_set_ocean.  Errors: SP_EINVAL. */
sp_status sp_gdem_set_ocean(sp_gdem* g, double u0, double v0, int32_t nmodes, const double* kx,
                            const double* ky, const double* au, const double* av, const double* phase);
/* n >= 1 floes from host arrays of length n (copied; omega and theta may be
 * NULL).  Floe i keeps index i in sp_gdem_read_floes.  Synchronises.
 * Errors: SP_EINVAL (r <= 0, h <= 0, r_max >= min(lx, ly) / 4), SP_ENOMEM. */
sp_status sp_gdem_set_floes(sp_gdem* g, int64_t n, const uint32_t* xi, const uint32_t* yi,
                            const float* u, const float* v, const float* omega, const float* theta,
                            const float* r, const float* h);
/* nsteps fine steps of size dt.  Asynchronous.  Errors: SP_EINVAL, SP_ESTATE. */
sp_status sp_gdem_step(sp_gdem* g, double dt, int64_t nsteps);
/* Floe state into caller-owned host arrays of length n in input order (any
 * may be NULL).  Synchronises; returns a latched device fault. */
sp_status sp_gdem_read_floes(sp_gdem* g, uint32_t* xi, uint32_t* yi, float* u, float* v, float* omega,
                             float* theta, float* r);
/* The SP_NMOM statistics (order as SP_MOMENTS_DEM, drag at the current state)
 * of every cell of an nxc x nyc coarse grid over the domain into out
 * [nyc * nxc][SP_NMOM] (cell iy * nxc + ix); a floe counts in the cell holding
 * its centre.  Synchronises.  Errors: SP_EINVAL (nxc, nyc < 1, more than 2^26
 * cells, null out), SP_ESTATE. */
sp_status sp_gdem_coarse_moments(sp_gdem* g, int32_t nxc, int32_t nyc, double* out);
/* Contacts summed over steps (each pair once per step), steps taken and the
 * sub-bins per side.  Synchronises. */
sp_status sp_gdem_get_stats(sp_gdem* g, int64_t* contacts, int64_t* steps, int32_t* bins_x,
                            int32_t* bins_y);
/* Debug/test call: the floe indices (those of sp_gdem_set_floes) in the
 * context's current order, grouped by the sub-bins of the positions at the
 * last re-binning; the starts of those sub-bins in that order
 * [bins_x * bins_y + 1]; and how many sub-bins and coarse cells gathered their
 * floes by scanning every floe (a floe that moved more than one sub-bin since
 * the previous grouping).  Any output may be NULL.  Synchronises. */
sp_status sp_gdem_read_order(sp_gdem* g, int32_t* ids, int32_t* starts, int64_t* fallbacks);

#ifdef __cplusplus
}
#endif

#endif /* SPDEM_H */
