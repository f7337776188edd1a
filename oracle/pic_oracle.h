/*
 * FP64 CPU oracle for the energy-conserving (EC) electrostatic PIC/MCC step
 * of Wang, Sun, Jiang & Kong, "On the energy conservation electrostatic
 * PIC/MC simulating" (arXiv:1310.5284).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a plain, slow, obviously-correct
 * restatement of the method used to check the GPU library.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header, table or constant with the GPU path.
 *
 * Every floating-point quantity is double precision.  Positions are kept as
 * xi = x / dx (cell units, node g sits at xi = g, cell j spans [j, j+1)).
 * Velocities are in m/s, fields in V/m, charge densities in C/m^3 and areal
 * macro-particle weights in physical particles per macro-particle per m^2.
 *
 * Functions whose result is not pinned by an independent check say so in
 * their comment ("parity unpinned").
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_DIRICHLET = 0, ORC_BC_PERIODIC = 1 };
enum { ORC_EXPLICIT = 0, ORC_IMPLICIT = 1 };
/* EC: Eqs. (2)-(3) with m = 1 (S_1 deposit, S_0 gather of the half-grid
 * field); MC: S_1 deposit, S_1 gather of the nodal field; EC2: Eqs. (2)-(3)
 * with m = 2 read as spline degree (S_2 deposit, S_1 gather of the half-grid
 * field); its direct-implicit solve takes the tridiagonal susceptibility
 * operator of orc_chi_operator_ec2 (orc_solve_chi_tridiag). */
enum { ORC_GATHER_EC = 0, ORC_GATHER_MC = 1, ORC_GATHER_EC2 = 2 };
enum { ORC_ELASTIC = 0, ORC_EXCITATION = 1, ORC_IONIZATION = 2, ORC_CHARGE_EXCHANGE = 3 };

typedef struct {
    int32_t n_cells;        /* N cells, N+1 nodes                                  */
    int32_t bc;             /* ORC_BC_*                                            */
    int32_t scheme;         /* ORC_EXPLICIT or ORC_IMPLICIT (D1, beta = 1/2)       */
    int32_t gather;         /* ORC_GATHER_EC (Eq. 3), ORC_GATHER_MC (CIC), EC2     */
    int32_t collisions;     /* 0 / 1                                               */
    /* Ion subcycling K (explicit scheme; 0 or 1: none): ions are pushed,
     * absorbed and collided only in steps n with n % K == 0, with the time
     * step K dt (null-collision probability 1 - exp(-nu_max K dt)); in the
     * other steps they stand and keep their charge on the grid. */
    int32_t ion_subcycle;
    double gap_m;           /* L                                                   */
    double dt_s;
    int64_t step0;          /* absolute index of the first step to take            */
    double rf_volts;        /* V(t) = V0 sin(2 pi f t) on the node at x = 0        */
    double rf_freq_hz;
    double gas_density_m3;
    double gas_temp_K;
    double gas_mass_kg;     /* neutral mass (elastic recoil, neutral velocities)   */
    double background_rho;  /* fixed uniform charge density, C/m^3                 */
    double opal_B_eV;       /* energy-sharing parameter of ionization              */
    uint64_t seed;          /* Philox key                                          */
    /* NULL: N equal cells of L/N.  Otherwise the N cell widths (m, summing to
     * L; electrodes only): a nonuniform grid, finer in the
     * sheaths.  Positions stay logical (cell index + offset in the cell). */
    const double* cell_dx_m;
} orc_case;

/* Per-step energy and particle ledger (all energies J/m^2). */
typedef struct {
    double K_before[2];     /* kinetic energy of the particles alive at step start  */
    double K_after[2];      /* kinetic energy at n+1/2 of the particles alive after */
    double work[2];         /* sum over pushed particles of the field work          */
    double coll_dK[2];      /* kinetic-energy change from collisions incl. children */
    double absorbed_K[2][2];/* [species][electrode 0 = x=0, 1 = x=L]                */
    double WE;              /* field energy sum 1/2 eps0 E^2 dx of this step's solve*/
    int64_t absorbed_n[2][2];
    int64_t n_coll[2][4];   /* real collisions by process kind                      */
    int64_t n_candidates[2];
    int64_t n_created[2];
    int64_t n_over_table[2];
} orc_ledger;

typedef struct orc_sim orc_sim;

/* ---- building blocks, used by the step and called directly by the pins ---- */

/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* (2*(r>>9)+1) * 2^-24: an odd multiple of 2^-24 in (0,1). */
double orc_u01(uint32_t r);

/* Eq. (2) with the linear spline S_1: Q[g] += S_1(g - xi_p) (dimensionless).
 * Q has N+1 entries; periodic mode folds node N onto node 0. */
void orc_deposit_linear(int32_t N, int32_t periodic, int64_t n, const double* xi,
                        double* Q);
/* Particle count per cell (floor(xi)) for the susceptibility. */
void orc_count_cells(int32_t N, int64_t n, const double* xi, double* cnt);

/* Field solves.  rho has N+1 node values; chi (may be NULL) has N cell values
 * chi_{j+1/2}.  Output phi (N+1) and the staggered field E_{j+1/2} (N). */
void orc_solve_dirichlet(int32_t N, double dx, const double* rho, const double* chi,
                         double phi0, double phiN, double* phi, double* E);
/* Dirichlet solve on a nonuniform grid of cell widths w[N]:
 *   (eps0 (1+chi_{g-1}) / w_{g-1}) (phi_g - phi_{g-1})
 *     - (eps0 (1+chi_g) / w_g) (phi_{g+1} - phi_g) = sigma_g,  g = 1..N-1,
 * sigma_g the charge per unit area of node g (C/m^2);
 * E_{j+1/2} = (phi_j - phi_{j+1}) / w_j. */
void orc_solve_dirichlet_nu(int32_t N, const double* w, const double* sigma, const double* chi,
                            double phi0, double phiN, double* phi, double* E);
void orc_solve_periodic(int32_t N, double dx, const double* rho, const double* chi,
                        double* phi, double* E);

/* Eq. (3) gathers at one particle. */
double orc_gather_ec(int32_t N, const double* E, double xi);
double orc_gather_mc(int32_t N, int32_t periodic, const double* E, double xi);
/* MC gather on a nonuniform grid of cell widths w[N] (electrodes): linear
 * interpolation of the nodal field (phi_{g-1} - phi_{g+1}) / (w_{g-1} + w_g). */
double orc_gather_mc_nu(int32_t N, const double* w, const double* E, double xi);
/* Eq. (3) with m = 2 on a nonuniform grid of widths w[N] (electrodes): minus
 * the derivative of the quadratic deposit's field energy with respect to the
 * physical position, (1/w_c) sum_h E_{h+1/2} w_h S_1(xi - (h + 1/2)). */
double orc_gather_ec2_nu(int32_t N, const double* w, const double* E, double xi);
/* Eq. (2) with the quadratic spline S_2 (degree 2, support 3 cells): a
 * particle at xi with nearest node i = floor(xi + 1/2) and d = xi - i gives
 * (1/2 - d)^2 / 2, 3/4 - d^2, (1/2 + d)^2 / 2 to nodes i-1, i, i+1.  Nodes
 * beyond an electrode fold into it (Dirichlet); periodic nodes wrap. */
void orc_deposit_quadratic(int32_t N, int32_t periodic, int64_t n, const double* xi,
                           double* Q);
/* Eq. (3) with m = 2: S_1 interpolation of the half-grid field E_{j+1/2}
 * (values at the cell centres); beyond an electrode the half-grid field is 0
 * (the counterpart of folding the charge into the electrode node). */
double orc_gather_ec2(int32_t N, int32_t periodic, const double* E, double xi);
/* Susceptibility weights of the direct-implicit scheme with m = 2, one per
 * cell centre.  Displacing particle p by d_p moves, with the S_2 deposit,
 * the charge flux S_1(x_p - x_h) d_p through centre h; the D1 correction d_p
 * is proportional to the S_1 gather sum_h' S_1(x_p - x_h') E_h' (no field
 * beyond an electrode).  The exact operator is therefore proportional to the
 * tridiagonal M_hh' = sum_p S_1(x_p - x_h) S_1(x_p - x_h'); these weights
 * are its row sums, w_h = sum_p S_1(x_p - x_h) sum_h' S_1(x_p - x_h'), the
 * diagonal approximation of the implicit m = 2 solve (h, h' over the N
 * centres of the grid, wrapped when periodic). */
void orc_chi_weights_ec2(int32_t N, int32_t periodic, int64_t n, const double* xi, double* w);

/* The operator itself, M_hh' = sum_p S_1(x_p - x_h) S_1(x_p - x_h'): a
 * particle between centres a and a + 1 at fraction t from a adds (1 - t)^2
 * to diag[a], t^2 to diag[a + 1] and t (1 - t) to off[a], the coupling of
 * centres a and a + 1 (off[N - 1]: of centres N - 1 and 0, periodic only;
 * no centre beyond an electrode). */
void orc_chi_operator_ec2(int32_t N, int32_t periodic, int64_t n, const double* xi,
                          double* diag, double* off);

/* Field solve of the direct-implicit scheme with a tridiagonal
 * susceptibility (the m = 2 operator): Gauss's law between half-grid
 * points gives D_{j+1/2} = D0 + R_j, R_j = dx sum_{k=1..j} rho_k, and the
 * field solves eps0 (E_j + sum_j' X_jj' E_j') = D_{j+1/2} with X_jj = xd[j],
 * X_{j,j+1} = X_{j+1,j} = xo[j] (xo[N-1]: the wrap, periodic only).  D0 is
 * fixed by dx sum_j E_j = phi_0 - phi_N (phi_N = 0, or a periodic
 * potential with phi_0 = 0).  Two solves of (1 + X) (Thomas; periodic:
 * Gaussian elimination with partial pivoting of the dense matrix), for the
 * constant and for R. */
void orc_solve_chi_tridiag(int32_t N, int32_t periodic, double dx, const double* rho,
                           const double* xd, const double* xo, double phi0, double* phi,
                           double* E);

/* The same on a nonuniform grid (cell widths w, between electrodes; dx =
 * L/N, r_j = w_j / dx).  A particle's D1 displacement along the gathered
 * field, (1/w_c) sum_h E_h w_h S_1, moves it by that over w_c in the
 * logical coordinate, so the operator carries 1/r_c^2 of its cell c
 * (orc_chi_operator_ec2_nu) and acts on F_j = r_j E_j, which keeps it
 * symmetric: (1/r + X) F = (D0 + R) / eps0 with R_j = sum_{k=1..j} sigma_k
 * (charges per area) and dx sum_j F_j = phi_0 - phi_N. */
void orc_chi_operator_ec2_nu(int32_t N, const double* w, double dx, int64_t n,
                             const double* xi, double* diag, double* off);
void orc_solve_chi_tridiag_nu(int32_t N, const double* w, double dx, const double* sigma,
                              const double* xd, const double* xo, double phi0, double* phi,
                              double* E);

/* ---- the simulation object ---- */
orc_sim* orc_create(const orc_case* c);
void orc_destroy(orc_sim* s);
/* species 0 = electrons, 1 = ions.  Arrays are copied.  abar may be NULL;
 * wait (null-collision waiting times: the number of steps, >= 0, before the
 * particle's next candidacy) may be NULL: orc_prepare then draws them for a
 * first trial at step0. */
int orc_set_species(orc_sim* s, int32_t sp, double q, double m, double w, int64_t n,
                    const double* xi, const double* vx, const double* vy,
                    const double* vz, const double* abar, const uint64_t* id,
                    const int64_t* wait);
/* One collision process on a uniform energy grid e0 + k*de, k = 0..n-1. */
int orc_add_process(orc_sim* s, int32_t sp, int32_t kind, double threshold_eV,
                    double e0_eV, double de_eV, int32_t n, const double* sigma_m2);
/* Computes the null-collision frequencies and draws the waits of species
 * loaded without them; must follow the last add_process. */
int orc_prepare(orc_sim* s);
/* D1 start-up: with loaded (x_0, v_{-1/2}) and abar = 0 store the first
 * prediction x~_1 = x_0 + dt v_{-1/2}; particles predicted outside are removed. */
int orc_implicit_startup(orc_sim* s);
/* Deposit + field solve of the current state without moving anything. */
int orc_compute_fields(orc_sim* s);
/* Take n steps (scheme from the case).  Returns 0, or a negative error. */
int orc_step(orc_sim* s, int64_t n);
/* One step in which the gather uses the given field E (N values, V/m) instead
 * of depositing and solving: for checking a particle sample of a discharge
 * too large for the oracle against the field of the whole discharge. */
int orc_step_with_field(orc_sim* s, const double* E);

int64_t orc_count(const orc_sim* s, int32_t sp);
int64_t orc_step_index(const orc_sim* s);
void orc_get_species(const orc_sim* s, int32_t sp, double* xi, double* vx, double* vy,
                     double* vz, double* abar, uint64_t* id, int64_t* wait);
/* Fields of the most recent solve: rho (N+1), phi (N+1), E (N), chi (N),
 * Q per species (N+1, dimensionless deposit), cell counts per species (N). */
void orc_get_fields(const orc_sim* s, double* rho, double* phi, double* E, double* chi,
                    double* Qe, double* Qi, double* cnt_e, double* cnt_i);
void orc_get_ledger(const orc_sim* s, orc_ledger* out);
/* Cumulative per-cell field work (J/m^2) per species since creation (N each). */
void orc_get_heating(const orc_sim* s, double* he, double* hi);
double orc_numax(const orc_sim* s, int32_t sp);

/* ---- collision kernels exposed for the statistical pins ---- */
/* One step of the candidacy rule of particle id of species sp at `step` with
 * waiting time *wait (updated): returns 1 if the particle is a null-collision
 * candidate in this step (*wait was 0; the next wait is then drawn from u0
 * of draw 0), else 0 (*wait decremented).  Each particle is a candidate in
 * each step with probability P_null, independently (Vahedi & Surendra
 * 1995).  Waits are plain integers with no upper limit. */
int orc_mcc_wait_step(const orc_sim* s, int32_t sp, uint64_t id, int64_t step, int64_t* wait);
/* The wait of a particle whose first trial is at `step` (loaded without a
 * wait, or born by ionization in the step before): Geo0(P_null) from u0 of
 * draw 4 of its stream at `step`. */
int64_t orc_mcc_first_wait(const orc_sim* s, int32_t sp, uint64_t id, int64_t step);
/* Collision of one candidate with velocity v (m/s, in place): draw 0 gives
 * the process (u1) and the scattering angles (u2, u3).  Returns the process
 * kind that happened or -2 (null collision).
 * On ionization writes the ejected electron's velocity to ve and the new ion's
 * velocity to vi.  eps_over counts over-table energies. */
int orc_collide_one(orc_sim* s, int32_t sp, uint64_t id, int64_t step, double* v,
                    double* ve, double* vi, int* eps_over);

#ifdef __cplusplus
}
#endif
#endif
