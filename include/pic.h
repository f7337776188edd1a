/*
 * pic.h -- C-ABI of the MI355X (gfx950) hot path of the energy-conserving
 * (EC) electrostatic PIC/MCC method of Wang, Sun, Jiang & Kong,
 * arXiv:1310.5284 ("On the energy conservation electrostatic PIC/MC
 * simulating").
 *
 * One call advances every discharge ("case") held by a context by whole
 * steps.  A step of one case is, per particle: the field gathered from the
 * potential difference across the particle's own cell (Sec. II, Eq. (3) with
 * S_0 of the half-grid field; or the momentum-conserving CIC gather of the
 * conventional scheme, Sec. II scheme (1)), the leap-frog push (explicit) or
 * the D1 direct-implicit push (Sec. II schemes (3)-(4)), absorption at the
 * electrodes (Sec. III), null-collision Monte Carlo collisions against the
 * neutral gas (Sec. III), and linear-weighted charge deposition (Sec. II,
 * Eq. (2) with S_1) -- plus, per case, the FP64 field solve.
 *
 * Conventions
 *   - Cells j = 0..N-1 span [j dx, (j+1) dx), dx = gap / N; nodes g = 0..N.
 *     A particle position is an int32 cell index and a float offset in [0,1).
 *   - Species 0 is the electron species, species 1 the ion species, of every
 *     case.  Either may be empty.
 *   - All pointers passed in may be host or device pointers (the library
 *     copies with hipMemcpyDefault).  Nothing passed in is retained: every
 *     input array may be freed once the call returns.
 *   - Status: every int-returning call returns PIC_OK (0) or a negative
 *     PIC_E_* code and never throws.  pic_last_error() gives a text.
 *   - Threading: a context is used by one host thread at a time.  Step calls
 *     are asynchronous on the context's stream; pic_diagnostics synchronises
 *     it.  A device fault makes the context sticky-failed (PIC_E_STATE).
 */
#ifndef PIC_H
#define PIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PIC_OK = 0,
    PIC_E_INVAL = -1,      /* bad argument or configuration                    */
    PIC_E_NOMEM = -2,      /* device allocation failed                         */
    PIC_E_CAPACITY = -3,   /* particle capacity exceeded (children were lost)  */
    PIC_E_UNSTABLE = -4,   /* explicit case violates omega_p dt < 2 (Eq. (1))  */
    PIC_E_DEVICE = -5,     /* HIP runtime error                                */
    PIC_E_STATE = -6,      /* context unusable after an earlier failure        */
    PIC_E_DIVERGED = -7    /* non-finite field or energy detected              */
};

enum { PIC_BC_DIRICHLET_RF = 0, PIC_BC_PERIODIC = 1 };
/* PIC_IMPLICIT_D1: the D1 direct-implicit push (beta = 1/2) with the field
 * solve -d/dx(eps0 (1 + chi) dphi/dx) = rho~ of the predicted positions; the
 * susceptibility chi_{j+1/2} = beta dt^2/(eps0 dx) sum_s q_s^2 w_s/m_s N_{s,j}
 * counts the predicted particles of cell j (EC gather), or is the mean of
 * the two node values beta dt^2/eps0 sum_s q_s^2 w_s/m_s Q_{s,g}/V_g of the
 * linear node weights (MC gather; V_g = dx, dx/2 at an electrode node).
 * With PIC_GATHER_EC2, N_{s,j} is replaced by the row sum of the tridiagonal
 * operator sum_p S_1(x_p - x_j) S_1(x_p - x_j') over the cell centres (the
 * diagonal approximation of the exact susceptibility): a particle between
 * centres adds its two linear weights, one between an electrode and the
 * first centre the square of that centre's weight. */
enum { PIC_EXPLICIT = 0, PIC_IMPLICIT_D1 = 1 };
/* Weighting and interpolation (Sec. II, Eqs. (2)-(3)):
 * PIC_GATHER_EC: Eq. (2) with S_1 (linear deposit to the nodes) and Eq. (3)
 *   with S_0 (the half-grid field of the particle's own cell), m = 1;
 * PIC_GATHER_MC: S_1 deposit and S_1 interpolation of the nodal field
 *   (momentum-conserving);
 * PIC_GATHER_EC2: Eqs. (2)-(3) with m = 2 read as spline degree: quadratic
 *   S_2 deposit (weights beyond an electrode fold into its node) and S_1
 *   interpolation of the half-grid field (zero beyond an electrode). */
enum { PIC_GATHER_EC = 0, PIC_GATHER_MC = 1, PIC_GATHER_EC2 = 2 };
enum { PIC_ELASTIC = 0, PIC_EXCITATION = 1, PIC_IONIZATION = 2, PIC_CHARGE_EXCHANGE = 3 };

/* pic_init flags */
enum {
    /* skip the omega_p dt < 2 check of explicit cases (Eq. (1)) */
    PIC_FLAG_ALLOW_UNSTABLE = 1u << 0,
    /* particle arrays hold a state exported by pic_diagnostics(PIC_DIAG_STATE):
     * velocities in cells per step, abar in cells per step^2, and for implicit
     * cases the already-predicted position and velocity (no start-up push) */
    PIC_FLAG_INTERNAL_UNITS = 1u << 1
};

/* One discharge (Sec. III): planar gap, RF-driven electrode at x = 0 with
 * V(t) = rf_volts sin(2 pi rf_freq_hz t), grounded electrode at x = L; or a
 * periodic box.  t_n = n dt with n the absolute step index. */
typedef struct {
    int32_t n_cells;        /* N >= 2 and N <= PIC_MAX_CELLS                    */
    int32_t bc;             /* PIC_BC_*                                         */
    int32_t scheme;         /* PIC_EXPLICIT | PIC_IMPLICIT_D1 (beta = 1/2)      */
    int32_t gather;         /* PIC_GATHER_EC | PIC_GATHER_MC | PIC_GATHER_EC2   */
    int32_t collisions;     /* 0 / 1                                            */
    int32_t history_steps;  /* ledger rows kept on the device (ring), >= 0      */
    double gap_m;
    double dt_s;
    int64_t start_step;     /* absolute index of the next step                  */
    double rf_volts;
    double rf_freq_hz;
    double gas_density_m3;
    double gas_temp_K;
    double gas_mass_kg;     /* neutral mass: elastic recoil, neutral velocities */
    double background_rho;  /* fixed uniform charge density, C/m^3              */
    double opal_B_eV;       /* energy-sharing parameter of ionization (10 eV)   */
    uint64_t seed;          /* Philox4x32-10 key of this case                   */
    /* NULL: N equal cells of gap_m / N.  Otherwise N cell widths in metres
     * (host memory, read during pic_init only), positive and summing to
     * gap_m within 1e-9: a nonuniform grid, finer in the sheaths (the
     * multi-scale grid the conclusions propose).  PIC_BC_DIRICHLET_RF only;
     * PIC_GATHER_MC takes as nodal field the centred potential difference
     * over the node's two cells, PIC_GATHER_EC2 gathers minus the physical
     * gradient of the quadratic deposit's field energy; with PIC_IMPLICIT_D1
     * it solves the tridiagonal susceptibility for F_j = (w_j N / gap_m) E_j
     * and takes at most 4069 cells (the LDS of its moment words); other
     * combinations: PIC_E_INVAL.
     * Positions stay logical
     * (cell index + offset); velocities are in units of (gap_m / N) / dt_s. */
    const double* cell_dx_m;
    /* Ion subcycling K (PIC_EXPLICIT only; 0 or 1: none; at most 4096):
     * ions are pushed, absorbed and collided only in the steps n with
     * n % K == 0, with the time step K dt_s (null-collision probability
     * 1 - exp(-nu_max K dt_s)); in between they stand and their charge stays
     * on the grid. */
    int32_t ion_subcycle;
    int32_t reserved;       /* 0 */
} pic_case_config;

#define PIC_MAX_CELLS 4096

/* Null-collision waiting time of a particle (Vahedi & Surendra 1995, the
 * MCC of Sec. III): in every step every particle is a candidate with
 * probability P_null, independently; the library realises this Bernoulli
 * process by waiting times W ~ Geo0(P_null) = floor(ln u / ln(1 - P_null))
 * drawn from the particle's Philox stream, the number of non-candidate steps
 * before the next candidacy.  Word: count (bits 0..16) | PIC_WAIT_CAPPED for
 * a draw beyond the count range (when it runs out the step's trial is drawn
 * afresh). */
#define PIC_WAIT_MAX 0x1FFFFu
#define PIC_WAIT_CAPPED 0x20000u

/* One species of one case.  q_C, m_kg per physical particle; weight =
 * physical particles per macro-particle per m^2 of electrode area.
 * Positions: cell in [0, N), off in [0, 1).  Velocities in m/s unless
 * PIC_FLAG_INTERNAL_UNITS.  id: unique per species (the random stream of a
 * particle is keyed by (id, step)).  abar may be NULL (zero).  mcc_wait may
 * be NULL: every particle then draws its wait for a first trial at the start
 * step; a state exported by pic_diagnostics carries them for an exact
 * resume. */
typedef struct {
    double q_C, m_kg, weight;
    int64_t n;              /* particles given                                  */
    int64_t capacity;       /* slots reserved (>= n, <= 2^28 - 1024: the kernels
                               address 16-byte records with 32-bit offsets); ionization
                               appends children after the occupied slots       */
    const int32_t* cell;
    const float* off;
    const float* vx;
    const float* vy;
    const float* vz;
    const uint64_t* id;
    const float* abar;
    const uint32_t* mcc_wait;   /* waiting-time words (< 2^18) or NULL           */
} pic_species_init;

/* Cross-section table of one process on the uniform energy grid
 * e0_eV + k de_eV (k < n), linear in between, held constant outside.  For
 * electrons the energy is 1/2 m v^2; for ions 1/2 M g^2 with g the speed
 * relative to a neutral drawn from the gas Maxwellian.  A process with
 * threshold_eV > 0 cannot happen at or below its threshold.  All processes of
 * one species must share one grid; ions support PIC_CHARGE_EXCHANGE only.
 * The same tables serve every case of a context. */
typedef struct {
    int32_t species;
    int32_t kind;           /* PIC_ELASTIC ... PIC_CHARGE_EXCHANGE              */
    double threshold_eV;
    double e0_eV;
    double de_eV;
    int32_t n;
    const double* sigma_m2;
} pic_xsec;

/* Energy and particle ledger of one step of one case (energies J/m^2).
 * K_after[s] = K_before[s] + work[s] - sum absorbed_K[s][:] + coll_dK[s]. */
typedef struct {
    int64_t step;               /* index of the step this row describes         */
    double K_before[2];         /* kinetic energy at n-1/2                      */
    double K_after[2];          /* kinetic energy at n+1/2                      */
    double work[2];             /* field work on the particles                  */
    double coll_dK[2];          /* change from collisions, children included    */
    double absorbed_K[2][2];    /* [species][electrode: 0 at x=0, 1 at x=L]     */
    double WE;                  /* sum 1/2 eps0 E^2 dx of the solve this step used */
    int64_t absorbed_n[2][2];
    int64_t n_coll[2][4];       /* real collisions by process kind              */
    int64_t n_candidates[2];
    int64_t n_created[2];
    int64_t n_over_table[2];    /* candidates beyond the last table energy      */
    int64_t n_lost[2];          /* children dropped for lack of capacity        */
} pic_ledger;

/* pic_diagnostics what_mask bits */
enum {
    PIC_DIAG_FIELDS = 1u << 0,   /* rho, phi, E, chi, fixed-point deposits     */
    PIC_DIAG_LEDGER = 1u << 1,   /* last step's ledger (+ history if given)    */
    PIC_DIAG_STATE = 1u << 2,    /* particle export                            */
    PIC_DIAG_DENSITY = 1u << 3,  /* time-averaged node densities               */
    PIC_DIAG_HEATING = 1u << 4,  /* cumulative field work per cell             */
    PIC_DIAG_EEDF = 1u << 5      /* electron energy histogram                  */
};

/* Caller-owned output buffers (host or device pointers; NULL = skip). */
typedef struct {
    /* always filled */
    int64_t step;               /* absolute index of the next step              */
    int64_t n_particles[2];     /* live particles                               */
    int64_t n_slots[2];         /* occupied slots (live + not yet compacted)    */
    double vel_unit;            /* m/s per internal velocity unit (dx/dt)       */
    double acc_unit;            /* m/s^2 per internal abar unit (dx/dt^2)       */
    /* PIC_DIAG_FIELDS: the fields of the solve the next step uses */
    double* rho;                /* [N+1] C/m^3 (nonuniform grid: node charge per
                                 * area over half of each adjacent cell, the
                                 * whole end cell at an electrode)           */
    double* phi;                /* [N+1] V                                      */
    double* E;                  /* [N]   V/m at x_{j+1/2}                       */
    double* chi;                /* [N]   susceptibility chi_{j+1/2} (implicit), else 0 */
    int64_t* qfix[2];           /* [N+1] node deposits in units of 2^-24 particle */
    int64_t* cell_count[2];     /* [N]   particles per cell                     */
    /* PIC_DIAG_LEDGER */
    pic_ledger ledger;
    pic_ledger* history;        /* [history_cap] rows, oldest first             */
    int64_t history_cap;
    int64_t history_n;          /* rows written                                 */
    /* PIC_DIAG_STATE: live particles in slot order, internal units */
    int64_t state_cap[2];       /* capacity of the arrays below                 */
    int32_t* cell[2];
    float* off[2];
    float* vx[2];
    float* vy[2];
    float* vz[2];
    uint64_t* id[2];
    float* abar[2];
    uint32_t* mcc_wait[2];      /* null-collision waiting-time words            */
    /* PIC_DIAG_DENSITY: mean over sampled steps of the node density (m^-3):
     * the node's deposit over its volume, half of each adjacent cell (half a
     * cell at an electrode node; the widths of a nonuniform grid) */
    double* density[2];         /* [N+1]                                        */
    int64_t density_samples;
    /* PIC_DIAG_HEATING: sum over sampled steps of the field work per cell */
    double* heating[2];         /* [N]   J/m^2                                  */
    /* PIC_DIAG_EEDF: electron energy histogram summed over sampled steps */
    int32_t eedf_bins;          /* out: bins held by the context                */
    double eedf_bin_eV;         /* out: bin width                               */
    int64_t* eedf;              /* [eedf_bins]                                  */
    int64_t eedf_samples;
} pic_diag;

typedef struct pic_ctx pic_ctx;

/* Creates a context holding n_cases discharges.  species points to
 * 2*n_cases entries: [case][0 = electrons, 1 = ions].  hip_stream is a
 * hipStream_t that every launch goes to (NULL = a non-blocking stream that
 * the context creates and destroys); a batch holding both schemes also runs
 * the implicit cases' particle kernels on a second stream of the context's
 * own, together with the field solve of those cases; it waits on
 * hip_stream before its first step after a join, and hip_stream waits on it
 * before every compaction and graph replay and at the end of every step
 * call, so that work on hip_stream stays ordered with every call.  Validation: N range, dt > 0,
 * positions in range, ids present, tables consistent, capacity >= n, and for
 * explicit cases omega_p,max dt < 2 (Eq. (1)) unless PIC_FLAG_ALLOW_UNSTABLE.
 * On error *out is NULL and nothing is leaked. */
int pic_init(pic_ctx** out, int32_t n_cases, const pic_case_config* cases,
             const pic_species_init* species, const pic_xsec* xs, int32_t n_xs,
             void* hip_stream, uint32_t flags);

/* Advance every case of the context by n_steps.  Every case must be
 * PIC_EXPLICIT (resp. PIC_IMPLICIT_D1), else PIC_E_INVAL. */
int pic_step_explicit(pic_ctx* ctx, int64_t n_steps);
int pic_step_implicit(pic_ctx* ctx, int64_t n_steps);
/* Advance a mixed batch: each case by its own scheme, one launch per step. */
int pic_step(pic_ctx* ctx, int64_t n_steps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): pic_step
 * with no allocation of any kind.  Advances every case by n_steps exactly as
 * pic_step does (same kernels, bitwise the same results), with host launches
 * only (no graph replay, no timing events; pic_last_timing* then report 0)
 * and the kernels' per-step scratch -- the ledger partial rows and candidate
 * counts of every particle-pass workgroup and the compaction's bucket
 * histograms and cursors -- taken from a fixed device array of 2 MiB per
 * device instead of the context's buffers.  The array is shared by every
 * context and call on a device and keeps the last call's contents; calls
 * that overlap on one device (two host threads, or work on two streams in
 * flight at once) race on it and must not be made.  Synchronises the
 * context's stream.  Errors: PIC_E_INVAL if the schedule needs more scratch
 * than the array holds (rows x 164 bytes + 8 bytes per histogram bucket;
 * about 10 000 workgroups, i.e. choose a larger tile), or if the context's
 * device is not current; then those of pic_step. */
int pic_step_noalloc(pic_ctx* ctx, int64_t n_steps);

/* Synchronises the stream and copies what what_mask asks for, for one case,
 * into the caller's buffers.  Returns PIC_E_CAPACITY if a state buffer is
 * too small (out->n_particles then tells the size needed). */
int pic_diagnostics(pic_ctx* ctx, int32_t case_id, uint32_t what_mask, pic_diag* out);

/* Tuning and diagnostics cadence.  sort_every: steps between compaction and
 * cell sorting of the particle arrays (>= 1).  diag_every: steps between
 * samples of density, heating and EEDF (0 = off).  tile: particles per
 * workgroup (multiple of 256, <= 32768; 0 = keep). */
int pic_set_schedule(pic_ctx* ctx, int32_t sort_every, int32_t diag_every, int32_t tile);
/* Launch mode and kernel timing.  In both modes all cases of a scheme share
 * every launch.
 * graph = 0: every kernel is launched from the host.
 * graph = 1: one sort period (sort_every consecutive steps and the compaction
 *   that ends it) is captured into a HIP graph on first use and replayed
 *   whenever a call's remaining steps cover a whole period that starts at a
 *   period boundary; the other steps are launched from the host.  Steps with
 *   diagnostics samples (diag_every > 0), and periods longer than 1024 steps,
 *   are always launched from the host.  The graph is captured again after
 *   pic_set_schedule or pic_set_launch.  Requires a context stream other than
 *   the null stream (else PIC_E_INVAL).  Results are identical in both modes.
 * timing_every: HIP events bracket the particle and collision kernels of the
 *   steps whose index within the sort period is a multiple of timing_every
 *   (0 = no events; default 1).  Events recorded inside a replayed graph give
 *   the durations of the call's last replay; pic_last_timing* report the sum
 *   and count of the timed launches.
 * Errors: PIC_E_INVAL (bad values), PIC_E_STATE (failed context). */
int pic_set_launch(pic_ctx* ctx, int32_t graph, int32_t timing_every);
/* Store policy of the collision kernel for a candidate's new state (cell
 * word, velocity, record; implicit: offset and abar): 0 = the default cache
 * policy (lines stay cached for the next step's particle pass), 1 =
 * non-temporal stores (they do not evict what that pass reads).  Results are
 * identical; only the speed differs with the workload.  Default 0.
 * Errors: PIC_E_INVAL (not 0 or 1), PIC_E_STATE (failed context). */
int pic_set_store_policy(pic_ctx* ctx, int32_t nontemporal);
/* Autotuner of the launch schedule.  Runs real steps of the context (they
 * advance every case exactly as pic_step does, diagnostics cadence
 * included): first `steps_per_trial` steps at each tile of
 * tiles[0..n_tiles) at the current sort period, then whole sort periods
 * (at least steps_per_trial steps, from a period boundary) at each period of
 * sorts[0..n_sorts) with the fastest tile, then whole periods at the fastest
 * tile and period with store policy 0 and 1 (pic_set_store_policy).  Each
 * trial is timed by two HIP events around its launches on the context's
 * stream and follows two untimed steps at the new tile.  The fastest tile,
 * period and store policy are applied and the tile and period returned in
 * tile_out / sort_out (may be NULL).  ms_out (NULL or n_tiles + n_sorts + 2
 * entries, resp. of the defaults) receives the device milliseconds per step
 * of every trial, the two store policies last.
 * tiles == NULL: {1024, 2048, 4096, 8192, 16384, 32512}; sorts == NULL:
 * {16, 32, 64, 128} (the counts are then ignored).  Tiles must be positive
 * multiples of 256 up to 32512, periods positive.
 * Errors: PIC_E_INVAL (bad candidates), those of pic_step. */
int pic_autotune(pic_ctx* ctx, const int32_t* tiles, int32_t n_tiles, const int32_t* sorts,
                 int32_t n_sorts, int32_t steps_per_trial, int32_t* tile_out,
                 int32_t* sort_out, double* ms_out);
/* Zero the density, heating and EEDF accumulators of every case. */
int pic_reset_accumulators(pic_ctx* ctx);

/* Plain FP64 GPU form of the same method (fp64 absolute positions and
 * velocities, fp64 global-atomic deposit, no sort, one launch per phase),
 * used as the throughput comparison point: the explicit leap-frog and the D1
 * direct-implicit scheme (Sec. II schemes (1)-(4); beta = 1/2, the
 * susceptibility from fp64 cell counts (EC) or node weights (MC)), with the
 * null-collision MCC of Sec. III.  pic_fp64_reference_init copies the
 * context's current state (implicit cases: the predicted x~, v~ and abar)
 * and advances its own copy of it.  Cases with PIC_GATHER_EC or
 * PIC_GATHER_MC on uniform grids without subcycling only (else PIC_E_INVAL).
 * pic_fp64_reference_state: live particles, xi in cells, velocities in cells
 * per step (implicit: the predicted x~ and v~ = v_{n+1/2} + abar/2), abar in
 * cells per step^2 (0 for explicit cases); any output pointer may be NULL.  pic_fp64_reference_ledger: the
 * energy and particle ledger of the form's last step (as pic_ledger). */
int pic_fp64_reference_init(pic_ctx* ctx);
int pic_fp64_reference_step(pic_ctx* ctx, int64_t n_steps);
int pic_fp64_reference_state(pic_ctx* ctx, int32_t case_id, int32_t species, int64_t cap,
                             double* xi, double* vx, double* vy, double* vz, double* abar,
                             uint64_t* id, int64_t* n_out);
int pic_fp64_reference_ledger(pic_ctx* ctx, int32_t case_id, pic_ledger* out);

/* Measurement helper, independent of any context: allocates two device
 * buffers of `bytes` (a multiple of 16), copies one into the other `reps`
 * times with a plain streaming kernel on the null stream, frees them and
 * returns the mean milliseconds per copy.  Its FETCH_SIZE / WRITE_SIZE
 * counter readings calibrate the HBM traffic figures of the other kernels.
 * Errors: PIC_E_INVAL (bad sizes), PIC_E_NOMEM, PIC_E_DEVICE. */
int pic_copy_calibration(int64_t bytes, int32_t reps, double* ms_per_copy);

void pic_destroy(pic_ctx* ctx);
const char* pic_last_error(const pic_ctx* ctx);
/* Timing of the most recent pic_step* call: milliseconds of device time
 * spent in the timed launches of the particle kernel (HIP events on the
 * context's stream, see pic_set_launch) and the number of launches timed. */
int pic_last_timing(const pic_ctx* ctx, double* particle_kernel_ms, int64_t* launches);
/* The same for the collision kernel that follows each particle pass (the
 * null-collision MCC of the candidates the pass listed). */
int pic_last_timing_collide(const pic_ctx* ctx, double* collide_kernel_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif
