// Device-side data layout of the EC PIC/MCC hot path (gfx950).
//
// Internal units: positions as (int32 cell, float offset in [0,1)); velocities
// in cells per step (v dt/dx); accelerations in cells per step^2 (a dt^2/dx).
// Charge deposits are int64 fixed point with 2^-24 of a particle per unit:
// every block accumulates, per cell j, the count of particles in the cell and
// the sum of their right-node weights W = rint(off * 2^24); the node charge in
// particle units is then count_g * 2^24 - W_g + W_{g-1} (Eq. (2), linear S_1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int kBlock = 256;                 // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kFixBits = 24;                // deposit weight resolution
constexpr double kFixScale = 16777216.0;    // 2^24
constexpr unsigned long long kCountOne = 1ull << 40;  // packed LDS count unit
constexpr unsigned long long kWMask = kCountOne - 1;
constexpr int kMaxProc = 4;                 // electron processes per table row
constexpr int kEedfBins = 256;
constexpr int kMaxTile = 32767;             // keeps packed LDS counts < 2^16

// 16- and 8-byte vectors of uint32 (native vector types: loadable through
// global address-space pointers)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// One species of one case.  Particle pointers are swapped by the compaction.
// The streaming pass touches cell, off, vx (and abar); the collision inputs
// that only candidates need (id, vy, vz) form one 16-byte record per
// particle (x, y: id low and high words; z, w: vy and vz bits), so that a
// candidate touches one cache line instead of three.
struct Species {
    int32_t* cell;
    float* off;
    float* vx;
    u32x4* rec;
    float* abar;
    int32_t* cell2;
    float* off2;
    float* vx2;
    u32x4* rec2;
    float* abar2;
    int64_t capacity;
    double accel;        // cells/step^2 per (V/m): (q/m) dt^2 / dx
    double qw_dx;        // C/m^3 per particle of deposit: q w / dx
    double kin_unit;     // J/m^2 per unit v^2: m w (dx/dt)^2 / 2
    double chi_coef;     // beta dt^2 q^2 w / (m eps0 dx) per particle in a cell
    double dens_unit;    // m^-3 per particle of deposit: w / dx
    float eps_unit;      // eV per unit v^2: m (dx/dt)^2 / (2 e)
    float t_scale;       // table index per unit v^2: eps_unit / de
    float t_off;         // -e0 / de
    float t_max;         // n - 1
    float thr_v2[kMaxProc];  // process possible only for v^2 above this
    int32_t kind[kMaxProc];  // process kinds in table order (-1 unused)
    int32_t n_proc;
    uint32_t cand_thr;   // candidate iff (r >> 9) < cand_thr  (u0 < P_null)
    float vth_neutral;   // sqrt(k T_gas / M_gas) dt/dx (ions: neutral partner)
    float vth_newion;    // sqrt(k T_gas / M_ion) dt/dx (ion born by ionization)
    float recoil2;       // 2 m_e / M_gas (elastic energy loss)
    float opal_B;        // eV
    const float4* tab_e; // electron table: per energy point, sigma_k * sig_scale
    const float* tab_i;  // ion table (charge exchange), sigma * sig_scale
    float eedf_scale;    // EEDF bins per eV
    int32_t pad;
    double inv_log1mp;   // 1 / ln(1 - P_null) (geometric waiting times)
    // collision candidates of the running step, listed by k_step in the
    // region of each workgroup's chunk: slot, v_{n+1/2}, abar_n (implicit)
    int32_t* cq_idx;
    float* cq_vn;
    float* cq_ab;
    int32_t* cq_w;       // cell word of x_{n+1} (cell, waiting time)
    float* cq_o;         // offset of x_{n+1} (implicit)
    // electrons: upper bounds of sum_k n_g sigma_k v / nu_max (the scaled
    // table times the speed) over bins of bound_k table intervals
    const float* cbound;
    int32_t bound_k;
    int32_t pad2;
};

// Everything a kernel needs to know about one case.
struct Case {
    int32_t n_cells;
    int32_t bc;           // 0 Dirichlet RF, 1 periodic
    int32_t scheme;       // 0 explicit, 1 D1 implicit
    int32_t gather;       // 0 EC, 1 MC
    int32_t collisions;
    int32_t first_block;  // this case's first workgroup in the work table
    int32_t n_blocks;
    int32_t history_len;
    int32_t nonuniform;   // cell widths of their own (EC gather, electrodes)
    int32_t ion_sub;      // ion subcycling K >= 1: ions move in the steps n % K == 0
    double dx, dt;        // dx: the reference width L/N (velocity unit dx/dt)
    double rf_volts, rf_omega, rf_freq;
    double background_rho;
    uint32_t key0, key1;  // Philox key = seed
    Species sp[2];
    // per-case device arrays
    unsigned long long* dep_cnt[2];  // [N] particles per cell (accumulating)
    unsigned long long* dep_w[2];    // [N] sum of right-node weights
    // m = 2 implicit: the dual grid of the susceptibility (word e = k + 1
    // for the cell centres k, k + 1 on either side of a particle): counts and
    // summed fractions towards centre k + 1 (null otherwise)
    unsigned long long* chi_cnt[2];  // [N+1]
    unsigned long long* chi_w[2];    // [N+1]
    // m = 2 implicit on a nonuniform grid: the sums of P0 and of P2 over the
    // particles left of their nearest node (in the cell before it), so that
    // each side of a node can carry its own cell width (null otherwise)
    unsigned long long* chl_w0[2];   // [N+1]
    unsigned long long* chl_w2[2];   // [N+1]
    // nonuniform grid (null otherwise): r_c = dx / w_c for the moves and
    // w_c / dx for the solve
    float* cell_r;                   // [N]
    double* cell_wr;                 // [N]
    uint32_t* cell_run;              // [N] first | last << 16 cell of c's run of equal widths
    float* ehat[2];                  // [N] accel * E of the next step, per species
    double* E;                       // [N] V/m
    double* phi;                     // [N+1]
    double* rho;                     // [N+1]
    double* chi;                     // [N]
    long long* qfix[2];              // [N+1] node deposits (export)
    long long* ccount[2];            // [N] particles per cell (export)
    unsigned long long* dens_acc[2]; // [N+1] accumulated node deposits (diagnostics)
    double* heat_acc[2];             // [N] accumulated field work per cell (J/m^2)
    unsigned long long* eedf_acc;    // [kEedfBins]
    void* history;                   // pic_ledger ring
};

// Mutable per-case counters, written by the finalizing workgroup.
struct State {
    long long step;          // absolute index of the next step
    int32_t n_slots[2];      // occupied slots
    int32_t n_child[2];      // children appended during the running step
    int32_t n_live[2];
    int32_t flags;           // bit 0: non-finite field, bit 1: capacity
    double K[2];             // kinetic energy at the current half step (J/m^2)
    double WE[2];            // field energy of the field of step k, in slot k & 1
    long long dens_samples;
    long long eedf_samples;
    long long history_n;
    long long lost_total[2];
    long long sort_live[2];  // live counts found by the last compaction
    double sortK[2];         // exact kinetic energy found by the last compaction
    long long ledger_step;   // step whose ledger row is closed next
};

struct Work {
    int32_t c;   // case
    int32_t s;   // species
    int32_t b;   // workgroup index within (case, species)
    int32_t nb;  // workgroups of (case, species)
};

// A k_collide workgroup: round `round` of `rounds` over the candidates listed
// by k_step workgroup `step_blk` (the rounds take its blocks of kBlock
// candidates in turn).
struct CollideWork {
    int32_t step_blk;
    int32_t round;
    int32_t rounds;
    int32_t pad;
    Work w;   // the k_step workgroup's own entry (read with this one, not after it)
};

// Ledger partial sums of one workgroup, stored field-major: field f of
// workgroup b lives at pd[f * stride + b] (doubles) or pu[f * stride + b]
// (counters), so that a reduction over workgroups reads contiguous memory.
// Energies are in units of v^2 (cells per step squared) of the species.
enum PartD {
    PD_WORK = 0,      // [2] field work per species
    PD_COLL = 2,      // [2] collisional kinetic-energy change (children included)
    PD_ABSK = 4,      // [2][2] absorbed kinetic energy, species x electrode
    PD_V2 = 8,        // [2] compaction: exact sum of v^2 of live particles
    PD_N = 10
};
enum PartU {
    PU_ABS = 0,       // [2][2] absorbed particles
    PU_COLL = 4,      // [2][4] real collisions by process kind
    PU_CAND = 12,     // [2] candidates
    PU_CREATED = 14,  // [2] children created
    PU_OVER = 16,     // [2] candidates beyond the table
    PU_LOST = 18,     // [2] children lost for lack of capacity
    PU_N = 20
};

struct Params {
    Case* cases;
    State* state;
    const Work* work;
    double* pd;          // workgroup partials, PD_N fields x stride
    unsigned* pu;        // workgroup partials, PU_N fields x stride
    int32_t stride;      // workgroups in the work table
    int32_t n_cases;
    int32_t mode;        // kernel-specific
    int32_t* cand_n;     // candidates listed by each workgroup of the work table
    const CollideWork* cwork;   // k_collide work table
    int32_t nt_store;    // k_collide stores a candidate's new state non-temporally
};

constexpr int kBoundBins = 256;   // bins of the null-collision bound table
constexpr int kFinBlock = 1024;   // threads of the set-up solve and compaction workgroups
constexpr int kFinStep = 512;     // threads of a k_finalize workgroup (no register spill)
constexpr int kILP = 4;           // particles in flight per thread in k_step

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// Shared-memory layout of k_step for a case of N cells:
//   field[N+1] float  (EC: ehat of the cells; MC: nodal field)
//   dep[N+1] u64      (privatised deposit, count << 40 | summed weight)
//   DIAG: heat[N] float, eedf[kEedfBins] u32
// (dual: the susceptibility words of the m = 2 implicit scheme follow dep,
// on a nonuniform grid with the left-side sums of P0 and P2 after them;
// nu: the width ratios r_c of a nonuniform grid, N floats, and the runs of
// equal widths, N u32, follow those, unless the launch reads them from
// global memory: tables = false)
struct StepLds {
    size_t dep, dual, ratio, heat, eedf, total;
};
__host__ __device__ inline StepLds step_lds_layout(int N, bool diag, bool dual = false,
                                                   bool nu = false, bool tables = true)
{
    StepLds L;
    L.dep = align16(4 * ((size_t)N + 1));
    L.dual = L.dep + align16(8 * ((size_t)N + 1));   // N+1: the quadratic node grid
    L.ratio = L.dual + (dual ? (nu ? 3 : 1) * align16(8 * ((size_t)N + 1)) : 0);
    L.heat = L.ratio + (nu && tables ? 2 * align16(4 * (size_t)N) : 0);
    L.eedf = L.heat + (diag ? align16(4 * (size_t)N) : 0);
    L.total = L.eedf + (diag ? align16(4 * (size_t)kEedfBins) : 0);
    return L;
}

// Shared-memory layout of k_collide: dep[N+1] u64 (predicted positions of
// the implicit candidates) | (dual: susceptibility words[N+1] u64; on a
// nonuniform grid also the left-side sums, 2 x [N+1] u64) |
// eedf[kEedfBins] u32
struct CollideLds {
    size_t dual, eedf, total;
};
__host__ __device__ inline CollideLds collide_lds_layout(int N, bool dual, bool nu = false)
{
    CollideLds L;
    L.dual = align16(8 * ((size_t)N + 1));
    L.eedf = L.dual + (dual ? (nu ? 3 : 1) * align16(8 * ((size_t)N + 1)) : 0);
    L.total = L.eedf + align16(4 * (size_t)kEedfBins);
    return L;
}

// particles per thread moved together by k_compact_scatter
constexpr int kScatterILP = 4;

// The susceptibility of the implicit scheme with the m = 2 weighting has a
// dual grid of its own.
__host__ __device__ inline bool dual_chi(int scheme, int gather)
{
    return scheme == 1 && gather == 2;
}

}  // namespace pic
