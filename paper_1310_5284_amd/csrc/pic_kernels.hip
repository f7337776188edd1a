// HIP kernels of the EC PIC/MCC hot path for gfx950 (MI355X).
//
// One step of one case = one pass of k_step over the particle arrays of both
// species (gather, push, boundary, MCC, deposit), whose last-finishing
// workgroup then solves the FP64 field for the next step.  The method:
//   - charge weighting with the linear spline S_1 ........ Sec. II, Eq. (2)
//   - field interpolation with S_0 of the half-grid field  Sec. II, Eq. (3)
//     (EC), or CIC of the averaged nodal field (MC, scheme (1))
//   - explicit leap-frog / D1 direct-implicit push ....... Sec. II schemes (1)-(4)
//   - absorbing electrodes, RF bias, MCC with the gas .... Sec. III
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"
#include "pic_common.hpp"
#include "pic_device.hpp"

namespace pic {

// ---------------------------------------------------------------------------
// FP64 field solve of one case by one workgroup.
//
// Gauss's law between half-grid points, D_{j+1/2} - D_{j-1/2} = dx rho_j with
// D = eps0 (1 + chi) E, is integrated by a prefix sum: D_{j+1/2} = D_{1/2} +
// R_j, R_j = dx sum_{k=1..j} rho_k.  The one free constant follows from the
// boundary condition sum_j E_{j+1/2} dx = phi_0 - phi_N (V(t) on the driven
// electrode, or 0 for a periodic box).  chi = 0 is the Poisson solve of the
// explicit cycle; chi from the predicted cell counts the susceptibility-
// modified solve of the direct-implicit cycle.  O(log N) deep.
// ---------------------------------------------------------------------------
constexpr double kEps0 = 8.8541878128e-12;

template <int NT>
__device__ __forceinline__ void solve_case(Case* C, State* st, long long next_step,
                                           long long field_step, bool sample_density, double* S,
                                           double* red)
{
    constexpr int kPer = (PIC_MAX_CELLS + 1 + NT - 1) / NT;   // nodes per thread
    // register copy of the case: the stores below cannot alias it, so none
    // of its pointers is reloaded after a store
    const Case Cc = *C;
    const int N = Cc.n_cells, tid = threadIdx.x;
    const bool periodic = Cc.bc == 1;
    const bool implicit = Cc.scheme == 1;
    const double dx = Cc.dx;
    // X: chi_{j+1/2} of the cells (LDS, after the N+1 values of S); Y: chi
    // of the nodes (MC implicit: the susceptibility of the linear weights,
    // a half cell at an electrode node, averaged to the cells)
    double* X = S + N + 1;
    double* Y = X + N;
    const bool node_chi = implicit && Cc.gather == 1;
    // node g = tid + k NT needs the counts and weights of cells g and g-1
    const PIC_GLOBAL unsigned long long* dc[2] = {gp((const unsigned long long*)Cc.dep_cnt[0]),
                                                  gp((const unsigned long long*)Cc.dep_cnt[1])};
    const PIC_GLOBAL unsigned long long* dw[2] = {gp((const unsigned long long*)Cc.dep_w[0]),
                                                  gp((const unsigned long long*)Cc.dep_w[1])};
    // Nodes in batches of kB per thread; inside a batch every load is issued
    // before any result is used (unconditional loads from clamped indices,
    // selected afterwards, so that none waits behind a branch).
    constexpr int kB = 3;
    const double qs0 = Cc.sp[0].qw_dx / kFixScale, qs1 = Cc.sp[1].qw_dx / kFixScale;
    const double chi0 = Cc.sp[0].chi_coef, chi1 = Cc.sp[1].chi_coef;
    const double rho_bg = Cc.background_rho;
    const bool ec2 = Cc.gather == 2;   // quadratic deposit: node words
    for (int k0 = 0; k0 < kPer && k0 * NT <= N; k0 += kB) {
        long long cn[kB][2], wr[kB][2], wl[kB][2], qn[kB][2];
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            const int g = tid + (k0 + k) * NT;
            const int gg = (periodic && g == N) ? 0 : g;
            const int gl = gg > 0 ? gg - 1 : (periodic ? N - 1 : -1);
            const bool in = g <= N;
            const bool hr = in && gg < N, hl = in && gl >= 0;
            // m = 2 reads node words (N+1 of them); cell words otherwise
            const int ir = min(gg, ec2 ? N : N - 1), il = max(min(gl, N - 1), 0);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const long long c = (long long)dc[s][ir], r = (long long)dw[s][ir];
                const long long l = (long long)dw[s][il];
                cn[k][s] = hr ? c : 0;
                wr[k][s] = hr ? r : 0;
                wl[k][s] = hl ? l : 0;
                qn[k][s] = in ? r : 0;
            }
        }
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            const int g = tid + (k0 + k) * NT;
            if (g > N) continue;
            double rho = rho_bg, chin = 0.0;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const long long q =
                    ec2 ? qn[k][s] : cn[k][s] * (1ll << kFixBits) - wr[k][s] + wl[k][s];
                gp(Cc.qfix[s])[g] = q;
                if (sample_density) gatomic_add(gp(&Cc.dens_acc[s][g]), (unsigned long long)q);
                rho += (double)q * (s == 0 ? qs0 : qs1);
                chin += (double)q * (s == 0 ? chi0 : chi1);
            }
            if (node_chi) {
                const bool end = !periodic && (g == 0 || g == N);
                Y[g] = chin * ((end ? 2.0 : 1.0) / kFixScale);
            }
            gp(Cc.rho)[g] = rho;
            // R_j = dx sum_{k=1..j} rho_k: the summand of node 0 is zero
            S[g] = g == 0 ? 0.0 : rho * dx;
            if (g < N) {
                gp(Cc.ccount[0])[g] = cn[k][0];
                gp(Cc.ccount[1])[g] = cn[k][1];
                if (!node_chi) {
                    const double chi =
                        implicit ? chi0 * (double)cn[k][0] + chi1 * (double)cn[k][1] : 0.0;
                    X[g] = chi;
                    gp(Cc.chi)[g] = chi;
                }
            }
        }
    }
    lds_barrier();   // every deposit word has been read
    if (node_chi) {
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int j = tid + k * NT;
            if (j < N) {
                const double chi = 0.5 * (Y[j] + Y[j + 1]);
                X[j] = chi;
                gp(Cc.chi)[j] = chi;
            }
        }
        lds_barrier();
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int j = tid + k * NT;
        if (j <= N) {   // node N: the quadratic deposit's last node
            gp(Cc.dep_cnt[0])[j] = 0; gp(Cc.dep_cnt[1])[j] = 0;
            gp(Cc.dep_w[0])[j] = 0; gp(Cc.dep_w[1])[j] = 0;
        }
    }
    block_scan<double, NT>(S, N, red);             // S[j] = R_j
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int j = tid + k * NT;
        if (j < N) {
            const double kap = kEps0 * (1.0 + X[j]);
            a += S[j] / kap;
            b += 1.0 / kap;
        }
    }
    a = block_sum<double, NT>(a, red);
    b = block_sum<double, NT>(b, red);
    double V = 0.0;
    if (!periodic) {
        // V0 sin(2 pi f t) through the phase in cycles reduced to [0, 1)
        const double cyc = Cc.rf_freq * ((double)next_step * Cc.dt);
        V = Cc.rf_volts * sinpi(2.0 * (cyc - floor(cyc)));
    }
    const double D0 = (V / dx - a) / b;
    double we = 0.0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int j = tid + k * NT;
        if (j < N) {
            const double E = (D0 + S[j]) / (kEps0 * (1.0 + X[j]));
            X[j] = E;   // X now holds E
            gp(Cc.E)[j] = E;
            gp(Cc.ehat[0])[j] = (float)(Cc.sp[0].accel * E);
            gp(Cc.ehat[1])[j] = (float)(Cc.sp[1].accel * E);
            we += 0.5 * kEps0 * E * E * dx;
        }
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int j = tid + k * NT;
        if (j < N) S[j] = X[j];
    }
    we = block_sum<double, NT>(we, red);
    block_scan<double, NT>(S, N, red);
    const double phi0 = periodic ? 0.0 : V;
    if (tid == 0) gp(Cc.phi)[0] = phi0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int j = tid + k * NT;
        if (j < N) gp(Cc.phi)[j + 1] = phi0 - dx * S[j];
    }
    if (tid == 0) {
        st->WE[field_step & 1] = we;
        if (!isfinite(we)) atomicOr(&st->flags, 1);
        if (sample_density) st->dens_samples += 1;
    }
    lds_barrier();
}

// ---------------------------------------------------------------------------
// Ledger: the workgroup reduces the partials of the case's workgroups (fixed
// order: a strided per-thread sum, then a tree), then one thread writes the
// row and folds the appended children into the occupied slots.
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void reduce_partials(const double* pd_, const unsigned* pu_, int stride,
                                                int fb, int nb, double* sd, long long* su)
{
    // wavefront w sums the fields w, w + NT/64, ...: every lane strides over
    // the workgroup partials with kU loads in flight, then a wavefront tree
    constexpr int kU = 8;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const PIC_GLOBAL double* pd = gp(pd_);
    const PIC_GLOBAL unsigned* pu = gp(pu_);
    for (int f = wave; f < PD_N + PU_N; f += NT / 64) {
        if (f < PD_N) {
            double a[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) a[u] = 0.0;
            // unconditional loads from clamped indices keep all kU in flight
            const PIC_GLOBAL double* row = pd + (size_t)f * stride + fb;
            for (int b = lane; b < nb; b += 64 * kU)
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const double x = row[min(b + 64 * u, nb - 1)];
                    a[u] += b + 64 * u < nb ? x : 0.0;
                }
            double v = 0.0;
#pragma unroll
            for (int u = 0; u < kU; ++u) v += a[u];
            v = wave_sum(v);
            if (lane == 0) sd[f] = v;
        } else {
            // per-step counts of one case fit in 32 bits
            unsigned a = 0u;
            const PIC_GLOBAL unsigned* row = pu + (size_t)(f - PD_N) * stride + fb;
            for (int b = lane; b < nb; b += 64 * kU)
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const unsigned x = row[min(b + 64 * u, nb - 1)];
                    a += b + 64 * u < nb ? x : 0u;
                }
            a = wave_sum(a);
            if (lane == 0) su[f - PD_N] = (long long)a;
        }
    }
    lds_barrier();
}

// Called by every thread of the workgroup.  Thread 0 reads the case's state
// in one batch (no load waits behind a store), builds the row in LDS and
// writes the state back; the row is then copied out by many threads.
__device__ __forceinline__ void finish_ledger(Case* C, State* st, const double* sd, const long long* si)
{
    __shared__ pic_ledger row;
    __shared__ int ring;
    if (threadIdx.x == 0) {
        // fields of the state owned by the ledger (the field solve of the
        // same finalizer runs concurrently and owns step, WE[] and samples)
        const long long lstep = st->ledger_step;
        const double we = st->WE[lstep & 1];
        const double K0[2] = {st->K[0], st->K[1]};
        const int32_t slots[2] = {st->n_slots[0], st->n_slots[1]};
        const int32_t child[2] = {st->n_child[0], st->n_child[1]};
        const int32_t live[2] = {st->n_live[0], st->n_live[1]};
        const long long lost[2] = {st->lost_total[0], st->lost_total[1]};
        const long long hn = st->history_n;
        const double ku0 = C->sp[0].kin_unit, ku1 = C->sp[1].kin_unit;
        const long long cap0 = C->sp[0].capacity, cap1 = C->sp[1].capacity;
        const int hl = C->history_len;
        row.step = lstep;
        row.WE = we;
        bool finite = true;
        int flags = 0;
        for (int s = 0; s < 2; ++s) {
            const double ku = s == 0 ? ku0 : ku1;
            const long long cap = s == 0 ? cap0 : cap1;
            const double kb = K0[s];
            const double wk = sd[PD_WORK + s] * ku, cd = sd[PD_COLL + s] * ku;
            const double a0 = sd[PD_ABSK + 2 * s] * ku, a1 = sd[PD_ABSK + 2 * s + 1] * ku;
            const double ka = kb + wk - a0 - a1 + cd;
            row.K_before[s] = kb;
            row.work[s] = wk;
            row.coll_dK[s] = cd;
            row.absorbed_K[s][0] = a0;
            row.absorbed_K[s][1] = a1;
            row.K_after[s] = ka;
            st->K[s] = ka;
            finite = finite && isfinite(ka);
            row.absorbed_n[s][0] = si[PU_ABS + 2 * s];
            row.absorbed_n[s][1] = si[PU_ABS + 2 * s + 1];
            for (int k = 0; k < 4; ++k) row.n_coll[s][k] = si[PU_COLL + 4 * s + k];
            row.n_candidates[s] = si[PU_CAND + s];
            row.n_created[s] = si[PU_CREATED + s];
            row.n_over_table[s] = si[PU_OVER + s];
            row.n_lost[s] = si[PU_LOST + s];
            st->n_live[s] = live[s] + (int32_t)(si[PU_CREATED + s] - si[PU_ABS + 2 * s] -
                                                si[PU_ABS + 2 * s + 1]);
            st->lost_total[s] = lost[s] + si[PU_LOST + s];
            const long long ns = (long long)slots[s] + child[s];
            st->n_slots[s] = (int32_t)(ns < cap ? ns : cap);
            if (ns > cap || si[PU_LOST + s] > 0) flags |= 2;
            st->n_child[s] = 0;
        }
        if (!finite) flags |= 1;
        if (flags) atomicOr(&st->flags, flags);
        st->history_n = hn + 1;
        st->ledger_step = lstep + 1;
        ring = hl > 0 ? 1 + (int)(hn % hl) : -1;
    }
    lds_barrier();
    constexpr int kW = (int)(sizeof(pic_ledger) / 8);
    const long long* src = (const long long*)&row;
    long long* h = (long long*)C->history;
    for (int k = threadIdx.x; k < kW; k += blockDim.x) {
        h[k] = src[k];
        if (ring > 0) h[(size_t)ring * kW + k] = src[k];
    }
}

// Per-workgroup accumulators of the rare events (LDS).
struct BlockAcc {
    double absK[2][2];
    double other_dK;          // kinetic energy of ion children (electron blocks)
    unsigned abs_n[2][2];
    unsigned n_coll[4];
    unsigned n_created[2];
    unsigned n_over;
    unsigned n_lost[2];
    int cmin, cmax;
};

// Momentum-conserving gather: linear interpolation of the nodal field (held
// in LDS, N+1 nodes) at offset o of cell c.
__device__ __forceinline__ float gather_mc(const float* en, int c, float o)
{
    return (1.0f - o) * en[c] + o * en[c + 1];
}

// Eq. (3) with m = 2 (spline degree): linear interpolation of the half-grid
// field (cell values eh[N], at the cell centres) at offset o of cell c; no
// half-grid field beyond an electrode, a periodic grid wraps.
__device__ __forceinline__ float gather_ec2(const float* eh, int N, bool periodic, int c, float o)
{
    const bool up = o >= 0.5f;
    const int k = up ? c : c - 1;            // half-grid point at or left of x
    const float t = up ? o - 0.5f : o + 0.5f;
    float e0, e1;
    if (periodic) {
        e0 = eh[k < 0 ? N - 1 : k];
        e1 = eh[k + 1 >= N ? 0 : k + 1];
    } else {
        e0 = k >= 0 ? eh[k] : 0.0f;
        e1 = k + 1 < N ? eh[k + 1] : 0.0f;
    }
    return (1.0f - t) * e0 + t * e1;
}

// Eq. (2) with m = 2: quadratic (S_2) weights of a particle at offset o of
// cell c, in units of 2^-24 particle: nearest node i = c or c + 1,
// d = c + o - i in [-1/2, 1/2); nodes i-1, i, i+1 take (1/2 - d)^2 / 2,
// 3/4 - d^2, (1/2 + d)^2 / 2, the middle one as the exact complement.
__device__ __forceinline__ int quad_weights(int c, float o, uint32_t w[3])
{
    const bool up = o >= 0.5f;
    const float d = up ? o - 1.0f : o;
    const float a = 0.5f - d, b = 0.5f + d;
    w[0] = __float2uint_rn(0.5f * a * a * 16777216.0f);
    w[2] = __float2uint_rn(0.5f * b * b * 16777216.0f);
    w[1] = (1u << 24) - w[0] - w[2];
    return c + (up ? 1 : 0);
}

// A node index of the quadratic weights: folded into the electrode beyond
// which it lies (Dirichlet), wrapped (periodic).
__device__ __forceinline__ int fold_node(int g, int N, bool periodic)
{
    if (periodic) return g < 0 ? g + N : (g >= N ? g - N : g);
    return min(max(g, 0), N);
}

// Quadratic deposit of one particle per lane into a privatised node grid
// (N+1 words): weights in the low 40 bits; the particle's cell count rides on
// the word of node c (always one of the three).  Called by whole wavefronts.
// sorted: when every depositing lane is in one cell (cell-sorted ions), the
// lanes on each side of the cell centre share their three nodes, and their
// weights are summed across the wavefront before one atomic per node.
__device__ __forceinline__ void deposit_quad(unsigned long long* dep, bool want, int c, float o,
                                             int N, bool periodic, int& lo, int& hi,
                                             bool sorted = false)
{
    uint32_t w[3] = {0u, 0u, 0u};
    int i = c;
    if (want) i = quad_weights(c, o, w);
    if (sorted) {
        const unsigned long long m = __ballot(want);
        if (m == 0ull) return;
        const int lane = threadIdx.x & 63;
        const int leader = __ffsll((long long)m) - 1;
        const int cl = __builtin_amdgcn_readlane(c, leader);
        if (__ballot(want && c != cl) == 0ull) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const bool mine = want && (i == cl + side);
                const unsigned long long mg = __ballot(mine);
                if (mg == 0ull) continue;
                const int gl = __ffsll((long long)mg) - 1;
                uint32_t t[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) t[k] = wave_total_u32(mine ? w[k] : 0u);
                if (lane == gl) {
                    const int i0 = cl + side;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const int g0 = i0 - 1 + k;
                        const int g = fold_node(g0, N, periodic);
                        atomicAdd(&dep[g], (unsigned long long)t[k] +
                                               (g0 == cl ? (unsigned long long)__popcll(mg) *
                                                               kCountOne : 0ull));
                        range_note(lo, hi, g);
                    }
                }
            }
            return;
        }
    }
    if (!want) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int g0 = i - 1 + k;
        const int g = fold_node(g0, N, periodic);
        atomicAdd(&dep[g], (unsigned long long)w[k] + (g0 == c ? kCountOne : 0ull));
        range_note(lo, hi, g);
    }
}

// Nodal field of node g from the cell fields of one species: the mean of the
// two adjacent cells; the electrodes take the field of their own cell, a
// periodic grid wraps.
__device__ __forceinline__ float nodal_field(const PIC_GLOBAL float* eh, int N, bool periodic,
                                             int g)
{
    if (periodic) {
        const int gl = g == 0 ? N - 1 : g - 1;
        const int gr = g == N ? 0 : g;
        return 0.5f * (eh[gl] + eh[gr]);
    }
    if (g == 0) return eh[0];
    if (g == N) return eh[N - 1];
    return 0.5f * (eh[g - 1] + eh[g]);
}

__device__ __forceinline__ unsigned long long packw(float o)
{
    return kCountOne + (unsigned long long)__float2uint_rn(o * 16777216.0f);
}

// ---------------------------------------------------------------------------
// Collision of one candidate (null-collision MCC, Vahedi & Surendra 1995).
// Returns the process kind or -2 (null).  Velocities in cells/step.  S is the
// workgroup's register copy of the species constants; only constant indices
// go into its per-process arrays.
// ---------------------------------------------------------------------------
struct Child {
    float vx, vy, vz;
    float ix, iy, iz;   // new ion
    uint64_t ide, idi;
};

// An ionization queued by k_collide: the parent's slot, x_{n+1} (cell; the
// offset for implicit lists) and the pair it creates.
struct ChildEv {
    int32_t parent, cell;
    float off, pad;
    Child ch;
};
constexpr int kChildQ = 128;   // queued ionizations per k_collide workgroup

__device__ __forceinline__ int collide_electron(const Species& S, const float* bound, uint4 r0,
                                                uint64_t id, uint32_t step, uint32_t k0,
                                                uint32_t k1, float& vx, float& vy, float& vz,
                                                bool& over, Child& ch)
{
    const float v2 = vx * vx + vy * vy + vz * vz;
    const float vm = sqrtf(v2);
    const float t = fmaf(v2, S.t_scale, S.t_off);
    over = t > S.t_max;
    const float tc = fminf(fmaxf(t, 0.0f), S.t_max);
    const int k = min((int)tc, (int)S.t_max - 1);
    // a u1 above the bound of the energy bin is a null collision for certain:
    // decided without the table (the full comparison below would agree)
    if (!over && u01(r0.y) >= bound[min(k / S.bound_k, kBoundBins - 1)]) return -2;
    const float f = tc - (float)k;
    const PIC_GLOBAL float* tab = gp((const float*)S.tab_e) + 4 * k;
    float sg[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) sg[p] = fmaf(f, tab[4 + p] - tab[p], tab[p]);
    const float u1 = u01(r0.y);
    int kind = -2;
    float thr = 0.0f;
    float cum = 0.0f;
#pragma unroll
    for (int p = 0; p < kMaxProc; ++p) {
        if (p < S.n_proc && kind == -2) {
            const float sp = v2 > S.thr_v2[p] ? sg[p] : 0.0f;
            cum += sp * vm;
            if (u1 < cum) {
                kind = S.kind[p];
                thr = S.thr_v2[p];
            }
        }
    }
    if (kind == -2) return -2;
    float dx, dy, dz;
    iso_dir(u01(r0.z), u01(r0.w), dx, dy, dz);
    if (kind == PIC_ELASTIC) {
        const float cchi = vm > 0.0f ? (vx * dx + vy * dy + vz * dz) / vm : 0.0f;
        const float sp = sqrtf(v2 * (1.0f - S.recoil2 * (1.0f - cchi)));
        vx = sp * dx; vy = sp * dy; vz = sp * dz;
    } else if (kind == PIC_EXCITATION) {
        const float sp = sqrtf(fmaxf(v2 - thr, 0.0f));
        vx = sp * dx; vy = sp * dy; vz = sp * dz;
    } else if (kind == PIC_IONIZATION) {
        const uint4 r1 = philox((uint32_t)id, (uint32_t)(id >> 32), step, 1u, k0, k1);
        const uint4 r3 = philox((uint32_t)id, (uint32_t)(id >> 32), step, 3u, k0, k1);
        const float B = S.opal_B;
        const float avail = fmaxf(v2 - thr, 0.0f) * S.eps_unit;   // eV
        const float eej = B * tanf(u01(r1.x) * atanf(avail / (2.0f * B)));
        const float esc = fmaxf(avail - eej, 0.0f);
        const float s1 = sqrtf(esc / S.eps_unit);
        vx = s1 * dx; vy = s1 * dy; vz = s1 * dz;
        float ex, ey, ez;
        iso_dir(u01(r1.y), u01(r1.z), ex, ey, ez);
        const float s2 = sqrtf(eej / S.eps_unit);
        ch.vx = s2 * ex; ch.vy = s2 * ey; ch.vz = s2 * ez;
        float n1, n2, n3, n4;
        box_muller(u01(r3.x), u01(r3.y), n1, n2);
        box_muller(u01(r3.z), u01(r3.w), n3, n4);
        ch.ix = S.vth_newion * n1; ch.iy = S.vth_newion * n2; ch.iz = S.vth_newion * n3;
        ch.ide = child_id(id, step, 0u, k0, k1);
        ch.idi = child_id(id, step, 1u, k0, k1);
    }
    return kind;
}

__device__ __forceinline__ int collide_ion(const Species& S, uint4 r0, uint64_t id, uint32_t step,
                                           uint32_t k0, uint32_t k1, float& vx, float& vy,
                                           float& vz, bool& over)
{
    const uint4 r2 = philox((uint32_t)id, (uint32_t)(id >> 32), step, (1u << 28) | 2u, k0, k1);
    float n1, n2, n3, n4;
    box_muller(u01(r2.x), u01(r2.y), n1, n2);
    box_muller(u01(r2.z), u01(r2.w), n3, n4);
    const float wx = S.vth_neutral * n1, wy = S.vth_neutral * n2, wz = S.vth_neutral * n3;
    const float gx = vx - wx, gy = vy - wy, gz = vz - wz;
    const float g2 = gx * gx + gy * gy + gz * gz;
    const float t = fmaf(g2, S.t_scale, S.t_off);
    over = t > S.t_max;
    const float tc = fminf(fmaxf(t, 0.0f), S.t_max);
    const int k = min((int)tc, (int)S.t_max - 1);
    const float f = tc - (float)k;
    const PIC_GLOBAL float* tab = gp(S.tab_i);
    const float a = tab[k], b = tab[k + 1];
    const float sg = g2 > S.thr_v2[0] ? fmaf(f, b - a, a) : 0.0f;
    if (u01(r0.y) < sg * sqrtf(g2)) {
        vx = wx; vy = wy; vz = wz;
        return PIC_CHARGE_EXCHANGE;
    }
    return -2;
}

// ---------------------------------------------------------------------------
// Children of an ionization: one electron and one ion per event, appended
// after the occupied slots (one atomic per wavefront and species).
// ---------------------------------------------------------------------------
// Reserve slots for the lanes with want = true; returns the slot, -1 when
// not wanted, -2 when the species is full.
__device__ __forceinline__ long long reserve_slot(bool want, PIC_GLOBAL int32_t* counter,
                                                  int base_slots, long long cap)
{
    const unsigned long long m = __ballot(want);
    if (m == 0) return -1;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    int b = 0;
    if (lane == leader) b = gatomic_add(counter, (int32_t)__popcll(m));
    b = __shfl(b, leader, 64);
    if (!want) return -1;
    const long long slot = (long long)base_slots + b + rank;
    return slot < cap ? slot : -2;
}

__device__ __forceinline__ void write_particle(const Species& S, long long slot, int c, float o,
                                               float vx, float vy, float vz, uint64_t id,
                                               uint32_t wait, bool implicit)
{
    gp(S.cell)[slot] = pack_cell(c, wait);
    gp(S.off)[slot] = o;
    gp(S.vx)[slot] = vx;
    gp(S.rec)[slot] = make_rec(id, vy, vz);
    if (implicit) gp(S.abar)[slot] = 0.0f;
}

// ---------------------------------------------------------------------------
// Deposit of one particle per lane into the privatised LDS grid (Eq. (2)).
// When every depositing lane of the wavefront lands in the same cell (the
// common case for cell-sorted ions) the weights are summed across the
// wavefront first and one LDS atomic is issued instead of 64 colliding ones.
// Called with every lane of the wavefront active.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void deposit_wave(unsigned long long* dep, bool want, int c, float o,
                                             int& lo, int& hi)
{
    const unsigned long long m = __ballot(want);
    if (m == 0ull) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    const int cl = __builtin_amdgcn_readlane(c, leader);
    if (__ballot(want && c != cl) == 0ull) {
        // at most 64 * 2^24 = 2^30
        const unsigned w = wave_total_u32(want ? __float2uint_rn(o * 16777216.0f) : 0u);
        if (lane == leader) {
            atomicAdd(&dep[cl], ((unsigned long long)__popcll(m) << 40) + (unsigned long long)w);
            range_note(lo, hi, cl);
        }
    } else if (want) {
        atomicAdd(&dep[c], packw(o));
        range_note(lo, hi, c);
    }
}

// Deposit of one particle straight into the case grids (ionization
// children, rare): linear (count and weight of its cell) or quadratic.
__device__ __forceinline__ void deposit_global(const Case* C, int s, int c, float o)
{
    PIC_GLOBAL unsigned long long* gcnt = gp(C->dep_cnt[s]);
    PIC_GLOBAL unsigned long long* gw = gp(C->dep_w[s]);
    if (C->gather == 2) {
        uint32_t w[3];
        const int i = quad_weights(c, o, w);
        for (int k = 0; k < 3; ++k)
            gatomic_add(&gw[fold_node(i - 1 + k, C->n_cells, C->bc == 1)],
                        (unsigned long long)w[k]);
    } else {
        gatomic_add(&gw[c], packw(o) & kWMask);
    }
    gatomic_add(&gcnt[c], 1ull);
}

// ---------------------------------------------------------------------------
// k_step: the particle pass of one step of every case in this launch.
// Workgroup = a contiguous chunk of one species of one case.  Per particle
// (explicit, leap-frog):
//   a = ehat[cell] (EC, Eq. (3)) or the interpolated nodal field (MC);
//   v += a;  x += v;  absorb at the electrodes or wrap;  deposit (Eq. (2));
//   null-collision candidacy by the particle's waiting time.
// Per particle (implicit, D1, beta = 1/2; stored x~, v~, abar):
//   a = ehat[cell of x~];  x = x~ + a/2;  v = v~ + a/2;  abar = (abar + a)/2;
//   absorb; candidacy; non-candidates predict v~' = v + abar/2,
//   x~' = x + v~', absorb and deposit x~'.
//
// The streaming loop issues the loads of kILP particles per thread together
// (indices past the chunk are clamped to its last slot and treated as dead).
// Candidates store x_{n+1} and are listed (slot, v_{n+1/2}, abar_n) in the
// region of the workgroup's chunk for k_collide (ballot + one LDS atomic per
// wavefront).  The deposit goes to a privatised LDS grid (one int64 per cell
// packs count and summed weight), flushed over the cell range the workgroup
// touched.  The workgroup's ledger partial is a row of plain stores.
// ---------------------------------------------------------------------------
template <int SCHEME, bool DIAG>
__global__ __launch_bounds__(kBlock) void k_step(Params P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ BlockAcc acc;
    __shared__ int s_ncand;
    constexpr bool kImp = SCHEME == 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int gblk = P.mode + (int)blockIdx.x;
    const Work w = P.work[gblk];
    Case* C = P.cases + w.c;
    State* st = P.state + w.c;
    const int N = C->n_cells;
    const int s = w.s;
    // particle arrays (addressed by 32-bit byte offsets from a scalar base)
    // and the constants of the pass, read before any store
    PIC_GLOBAL int32_t* __restrict__ cellp = gp(uniform_ptr(C->sp[s].cell));
    PIC_GLOBAL float* __restrict__ offp = gp(uniform_ptr(C->sp[s].off));
    PIC_GLOBAL float* __restrict__ vxp = gp(uniform_ptr(C->sp[s].vx));
    const PIC_GLOBAL u32x4* __restrict__ recp = gp(uniform_ptr((const u32x4*)C->sp[s].rec));
    PIC_GLOBAL float* __restrict__ abp = gp(uniform_ptr(C->sp[s].abar));
    PIC_GLOBAL int32_t* __restrict__ cq_idx = gp(uniform_ptr(C->sp[s].cq_idx));
    PIC_GLOBAL float* __restrict__ cq_vn = gp(uniform_ptr(C->sp[s].cq_vn));
    PIC_GLOBAL float* __restrict__ cq_ab = gp(uniform_ptr(C->sp[s].cq_ab));
    PIC_GLOBAL int32_t* __restrict__ cq_w = gp(uniform_ptr(C->sp[s].cq_w));
    PIC_GLOBAL float* __restrict__ cq_o = gp(uniform_ptr(C->sp[s].cq_o));
    const float eedf_k = C->sp[s].eps_unit * C->sp[s].eedf_scale;
    const double kin_unit = C->sp[s].kin_unit;
    const bool periodic = C->bc == 1;
    const bool mc = C->gather == 1;
    const bool ec2 = C->gather == 2;
    const bool coll = C->collisions != 0 && C->sp[s].n_proc > 0;

    const StepLds L = step_lds_layout(N, DIAG);
    float* eh = (float*)smem;
    unsigned long long* dep = (unsigned long long*)(smem + L.dep);
    float* heat = (float*)(smem + L.heat);
    unsigned* eedf = (unsigned*)(smem + L.eedf);
    {
        const PIC_GLOBAL float* ehg = gp(C->ehat[s]);
        if (mc) {
            for (int g = tid; g <= N; g += kBlock) eh[g] = nodal_field(ehg, N, periodic, g);
        } else {
#pragma unroll 8
            for (int j = tid; j < N; j += kBlock) eh[j] = ehg[j];
        }
    }
#pragma unroll 8
    for (int j = tid; j < N; j += kBlock) {
        dep[j] = 0ull;
        if (DIAG) heat[j] = 0.0f;
    }
    if (tid == 0) dep[N] = 0ull;   // node N of the quadratic deposit
    if (DIAG)
        for (int j = tid; j < kEedfBins; j += kBlock) eedf[j] = 0u;
    if (tid == 0) {
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                acc.absK[a][b] = 0.0;
                acc.abs_n[a][b] = 0u;
            }
        acc.cmin = kNoCell;
        acc.cmax = -1;
        s_ncand = 0;
    }
    lds_barrier();

    const int n = st->n_slots[s];
    int chunk = (n + w.nb - 1) / w.nb;
    chunk = (chunk + 63) & ~63;
    const int start = w.b * chunk;
    const int end = min(n, start + chunk);

    double work = 0.0;
    int lo = kNoCell, hi = -1;

    auto absorb = [&](int i, int e, float vxh, float vy, float vz) {
        atomicAdd(&acc.absK[s][e], (double)(vxh * vxh + vy * vy + vz * vz));
        atomicAdd(&acc.abs_n[s][e], 1u);
        stg(cellp, (uint32_t)i << 2, -1);
    };

    // The loads of a batch (kILP particles per thread) are issued together,
    // one batch ahead of its processing, so that a wavefront keeps loads in
    // flight while it computes.  Indices past the chunk are clamped to its
    // last slot (and treated as dead below); the batch after the last one
    // reloads that slot and is discarded.
    int32_t cn[kILP];   // cell words of the next batch
    float on[kILP], vnx[kILP], abx[kILP];
    auto load_batch = [&](int b0) {
#pragma unroll
        for (int k = 0; k < kILP; ++k) {
            const uint32_t j4 = (uint32_t)min(b0 + k * kBlock + tid, end - 1) << 2;
            cn[k] = ldg(cellp, j4);
            on[k] = ldg(offp, j4);
            vnx[k] = ldg(vxp, j4);
            abx[k] = kImp ? ldg(abp, j4) : 0.0f;
        }
    };
    if (start < end) load_batch(start);
    for (int base = start; base < end; base += kBlock * kILP) {
        int32_t c[kILP];   // cell words
        float o[kILP], v[kILP], ab[kILP];
#pragma unroll
        for (int k = 0; k < kILP; ++k) {
            c[k] = cn[k];
            o[k] = on[k];
            v[k] = vnx[k];
            ab[k] = abx[k];
        }
        load_batch(base + kBlock * kILP);

        float wk = 0.0f;
#pragma unroll
        for (int k = 0; k < kILP; ++k) {
            const int i = base + k * kBlock + tid;
            const uint32_t i4 = (uint32_t)i << 2;
            const int cc = i < end ? cell_of(c[k]) : -1;
            uint32_t wt = wait_of(c[k]);
            bool live = cc >= 0;
            float a = 0.0f;
            if (live) a = mc ? gather_mc(eh, cc, o[k])
                             : (ec2 ? gather_ec2(eh, N, periodic, cc, o[k]) : eh[cc]);
            float vn, vold, abn = 0.0f, o1;
            if (kImp) {
                vold = v[k] - 0.5f * ab[k];
                vn = v[k] + 0.5f * a;
                abn = 0.5f * (ab[k] + a);
                o1 = o[k] + 0.5f * a;
            } else {
                vold = v[k];
                vn = v[k] + a;
                o1 = o[k] + vn;
            }
            int c1 = cc;
            if (live) {
                const float dk = (vn - vold) * (vn + vold);
                wk += dk;
                if (DIAG) {
                    atomicAdd(&heat[cc], dk);
                    range_note(lo, hi, cc);
                }
                renorm(c1, o1);
                if (periodic) {
                    c1 %= N;
                    if (c1 < 0) c1 += N;
                } else if (c1 < 0 || c1 >= N) {
                    const u32x4 r = ldg(recp, i4 << 2);
                    absorb(i, c1 < 0 ? 0 : 1, vn, rec_vy(r), rec_vz(r));
                    live = false;
                }
            }
            // null-collision candidacy by waiting time: a count above zero is
            // a non-candidate step; at zero the particle is a candidate (or,
            // for a capped wait, its trial is still open: decided by k_collide)
            bool isc = false;
            if (live && coll) {
                const uint32_t cnt = wt & PIC_WAIT_MAX;
                if (cnt > 0) wt = (cnt - 1) | (wt & PIC_WAIT_CAPPED);
                else isc = true;
            }
            // non-candidates finish here; candidates store x_{n+1} (final
            // for the explicit scheme, which deposits it now)
            int c2 = c1;
            float o2 = o1, vst = vn;
            bool dep_now = false;
            uint32_t lflag = 0u;   // list flag of a candidate
            if (live && !isc) {
                if (kImp) {
                    vst = predict(c2, o2, vn, abn);
                    if (periodic) {
                        c2 %= N;
                        if (c2 < 0) c2 += N;
                    } else if (c2 < 0 || c2 >= N) {
                        const u32x4 r = ldg(recp, i4 << 2);
                        absorb(i, c2 < 0 ? 0 : 1, vn, rec_vy(r), rec_vz(r));
                        live = false;
                    }
                }
                if (live) {
                    stg(cellp, i4, pack_cell(c2, wt));
                    stg(offp, i4, o2);
                    stg(vxp, i4, vst);
                    if (kImp) stg(abp, i4, abn);
                    dep_now = true;
                    if (DIAG && s == 0) {
                        const u32x4 r = ldg(recp, i4 << 2);
                        const float ey = rec_vy(r), ez = rec_vz(r);
                        const float fb = (vn * vn + ey * ey + ez * ez) * eedf_k;
                        const int bin =
                            fb >= 1.0f ? min((int)fminf(fb, (float)kEedfBins), kEedfBins - 1) : 0;
                        atomicAdd(&eedf[bin], 1u);
                    }
                }
            } else if (live) {
                bool kept = false;
                if (kImp) {
                    // implicit: predicted as if the collision were a null one
                    // (most are) and deposited; k_collide keeps that, or
                    // undoes the deposit and predicts again after a real
                    // collision.  A prediction outside the gap is left to
                    // k_collide.
                    int cp = c1;
                    float op = o1;
                    const float vp = predict(cp, op, vn, abn);
                    if (periodic) {
                        cp %= N;
                        if (cp < 0) cp += N;
                    }
                    if (cp >= 0 && cp < N) {
                        stg(cellp, i4, pack_cell(cp, wt));
                        stg(offp, i4, op);
                        stg(vxp, i4, vp);
                        stg(abp, i4, abn);
                        c2 = cp;
                        o2 = op;
                        lflag = kPredDeposited;
                        kept = true;
                    }
                }
                if (!kept) {
                    stg(cellp, i4, pack_cell(c1, wt));
                    stg(offp, i4, o1);
                    // explicit: v_{n+1/2} stands unless k_collide finds a
                    // real collision (the store joins the coalesced stream)
                    if (!kImp) stg(vxp, i4, vn);
                }
                dep_now = !kImp || kept;
            }
            if (ec2)
                deposit_quad(dep, dep_now, c2, o2, N, periodic, lo, hi, s == 1);
            else
                deposit_wave(dep, dep_now, c2, o2, lo, hi);
            // list the candidates of this wavefront in the workgroup's region
            const bool enq = live && isc;
            const unsigned long long qm = __ballot(enq);
            if (qm) {
                int b0 = 0;
                if (lane == 0) b0 = atomicAdd(&s_ncand, (int)__popcll(qm));
                b0 = __builtin_amdgcn_readfirstlane(b0);
                if (enq) {
                    const int e = start + b0 + (int)__popcll(qm & ((1ull << lane) - 1ull));
                    const uint32_t e4 = (uint32_t)e << 2;
                    stg(cq_idx, e4, i);
                    stg(cq_vn, e4, vn);
                    stg(cq_w, e4, pack_cell(c1, wt | lflag));
                    if (kImp) {
                        stg(cq_ab, e4, abn);
                        stg(cq_o, e4, o1);
                    }
                }
            }
        }
        work += (double)wk;
    }

    // flush the privatised deposit over the touched cell range
    if (hi >= 0) {
        atomicMin(&acc.cmin, lo);
        atomicMax(&acc.cmax, hi);
    }
    lds_barrier();
    {
        PIC_GLOBAL unsigned long long* gcnt = gp(C->dep_cnt[s]);
        PIC_GLOBAL unsigned long long* gw = gp(C->dep_w[s]);
        const int cl = acc.cmin, chh = acc.cmax;
        for (int j = cl + tid; chh >= 0 && j <= chh; j += kBlock) {
            const unsigned long long p = dep[j];
            if (p) {
                gatomic_add(&gcnt[j], p >> 40);
                gatomic_add(&gw[j], p & kWMask);
            }
            if (DIAG) {
                const float h = heat[j];
                if (h != 0.0f) gatomic_add(gp(&C->heat_acc[s][j]), (double)h * kin_unit);
            }
        }
        if (DIAG && s == 0)
            for (int j = tid; j < kEedfBins; j += kBlock)
                if (eedf[j]) gatomic_add(gp(&C->eedf_acc[j]), (unsigned long long)eedf[j]);
    }
    // workgroup partial of the ledger (plain stores; k_collide adds the
    // collision terms of the same workgroup, k_finalize reduces)
    __shared__ double wsum[kWaves];
    work = wave_sum(work);
    if (lane == 0) wsum[wave] = work;
    lds_barrier();
    // one field per thread
    if (tid < PD_N + PU_N) {
        const size_t S_ = (size_t)P.stride;
        if (tid < PD_N) {
            double x = 0.0;
            if (tid == PD_WORK + s)
                for (int k = 0; k < kWaves; ++k) x += wsum[k];
            else if (tid >= PD_ABSK && tid < PD_ABSK + 4)
                x = acc.absK[(tid - PD_ABSK) >> 1][(tid - PD_ABSK) & 1];
            P.pd[(size_t)tid * S_ + gblk] = x;
        } else {
            const int f = tid - PD_N;
            const unsigned x = f >= PU_ABS && f < PU_ABS + 4
                                   ? acc.abs_n[(f - PU_ABS) >> 1][(f - PU_ABS) & 1] : 0u;
            P.pu[(size_t)f * S_ + gblk] = x;
        }
        if (tid == 0) P.cand_n[gblk] = s_ncand;
    }
}

// ---------------------------------------------------------------------------
// k_collide: the null-collision MCC (Vahedi & Surendra 1995) of the
// candidates that k_step listed: one or more workgroups (rounds) per k_step
// workgroup, one candidate per thread.  A candidate whose capped wait ran out
// first draws its trial; a candidate draws its next waiting time, the
// process (u1 of draw 0 against the cumulative n_g sigma_k v / nu_max) and
// the scattering; ionizations are queued in LDS and append their electron
// and ion after the loop.  Implicit candidates keep the prediction k_step
// made for a null collision, or after a real one undo its deposit, predict
// again and are absorbed or deposit (privatised LDS grid).  The collision
// terms of the ledger are added to the row of the k_step workgroup.
// ---------------------------------------------------------------------------
template <int SCHEME, bool DIAG>
__global__ __launch_bounds__(kBlock) void k_collide(Params P)
{
    const CollideWork cw = P.cwork[P.mode + (int)blockIdx.x];
    const int gblk = cw.step_blk;
    const int ncand = P.cand_n[gblk];
    if (cw.round * kBlock >= ncand) return;   // nothing in this round
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ BlockAcc acc;
    __shared__ Species S;
    __shared__ ChildEv cq[kChildQ];
    __shared__ int q_n;
    constexpr bool kImp = SCHEME == 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const Work w = P.work[gblk];
    Case* C = P.cases + w.c;
    State* st = P.state + w.c;
    const int N = C->n_cells;
    const int s = w.s;
    PIC_GLOBAL int32_t* __restrict__ cellp = gp(uniform_ptr(C->sp[s].cell));
    PIC_GLOBAL float* __restrict__ offp = gp(uniform_ptr(C->sp[s].off));
    PIC_GLOBAL float* __restrict__ vxp = gp(uniform_ptr(C->sp[s].vx));
    PIC_GLOBAL u32x4* __restrict__ recp = gp(uniform_ptr(C->sp[s].rec));
    PIC_GLOBAL float* __restrict__ abp = gp(uniform_ptr(C->sp[s].abar));
    const PIC_GLOBAL int32_t* __restrict__ cq_w = gp(uniform_ptr((const int32_t*)C->sp[s].cq_w));
    const PIC_GLOBAL float* __restrict__ cq_o = gp(uniform_ptr((const float*)C->sp[s].cq_o));
    const PIC_GLOBAL int32_t* __restrict__ cq_idx =
        gp(uniform_ptr((const int32_t*)C->sp[s].cq_idx));
    const PIC_GLOBAL float* __restrict__ cq_vn = gp(uniform_ptr((const float*)C->sp[s].cq_vn));
    const PIC_GLOBAL float* __restrict__ cq_ab = gp(uniform_ptr((const float*)C->sp[s].cq_ab));
    const double inv_ion = C->sp[1].inv_log1mp;
    const long long cap0 = C->sp[0].capacity, cap1 = C->sp[1].capacity;
    PIC_GLOBAL unsigned long long* gdep_cnt = gp(uniform_ptr(C->dep_cnt[s]));
    PIC_GLOBAL unsigned long long* gdep_w = gp(uniform_ptr(C->dep_w[s]));
    // collision constants in LDS (stores to the particle arrays cannot alias them)
    for (int t = tid; t < (int)(sizeof(Species) / 4); t += kBlock)
        ((uint32_t*)&S)[t] = ((const uint32_t*)&C->sp[s])[t];
    const bool periodic = C->bc == 1;
    const uint32_t k0 = C->key0, k1 = C->key1;
    unsigned long long* dep = (unsigned long long*)smem;
    unsigned* eedf = (unsigned*)(smem + align16(8 * (size_t)N));
    __shared__ float lbound[kBoundBins];
    if (s == 0 && C->sp[0].n_proc > 0)
        for (int j = tid; j < kBoundBins; j += kBlock) lbound[j] = C->sp[0].cbound[j];
    if (kImp)
        for (int j = tid; j < N; j += kBlock) dep[j] = 0ull;
    if (DIAG)
        for (int j = tid; j < kEedfBins; j += kBlock) eedf[j] = 0u;
    if (tid == 0) {
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                acc.absK[a][b] = 0.0;
                acc.abs_n[a][b] = 0u;
            }
        acc.other_dK = 0.0;
        for (int k = 0; k < 4; ++k) acc.n_coll[k] = 0u;
        acc.n_created[0] = acc.n_created[1] = 0u;
        acc.n_over = 0u;
        acc.n_lost[0] = acc.n_lost[1] = 0u;
        acc.cmin = kNoCell;
        acc.cmax = -1;
        q_n = 0;
    }
    lds_barrier();

    const uint32_t step32 = (uint32_t)st->step;
    const int ns0 = st->n_slots[0], ns1 = st->n_slots[1];
    const int n = st->n_slots[s];
    int chunk = (n + w.nb - 1) / w.nb;
    chunk = (chunk + 63) & ~63;
    const int region = w.b * chunk;   // the candidate list of this workgroup
    const float eedf_k = S.eps_unit * S.eedf_scale;

    double cdk = 0.0;
    unsigned cand = 0u;
    int lo = kNoCell, hi = -1;

    auto absorb = [&](int i, int e, float vxh, float vy, float vz) {
        atomicAdd(&acc.absK[s][e], (double)(vxh * vxh + vy * vy + vz * vz));
        atomicAdd(&acc.abs_n[s][e], 1u);
        stg(cellp, (uint32_t)i << 2, -1);
    };

    // ionization children: electron and ion at the parent's x_{n+1};
    // implicit children are predicted from there with abar = 0; their
    // deposits are rare and go straight to the case grids.  Called by whole
    // wavefronts; lanes with ion_ev set emit one pair each.
    auto emit_children = [&](bool ion_ev, int c1, float o1, const Child& ch) {
        bool want_e = false, want_i = false;
        int ce = c1, ci = c1;
        float oe = o1, oi = o1;
        if (ion_ev) {
            const float ke = ch.vx * ch.vx + ch.vy * ch.vy + ch.vz * ch.vz;
            const float ki = ch.ix * ch.ix + ch.iy * ch.iy + ch.iz * ch.iz;
            cdk += (double)ke;
            atomicAdd(&acc.other_dK, (double)ki);
            atomicAdd(&acc.n_created[0], 1u);
            atomicAdd(&acc.n_created[1], 1u);
            want_e = want_i = true;
            if (kImp) {
                oe = o1 + ch.vx;
                renorm(ce, oe);
                oi = o1 + ch.ix;
                renorm(ci, oi);
                if (periodic) {
                    ce %= N; if (ce < 0) ce += N;
                    ci %= N; if (ci < 0) ci += N;
                } else {
                    if (ce < 0 || ce >= N) {
                        want_e = false;
                        const int eo = ce < 0 ? 0 : 1;
                        atomicAdd(&acc.absK[0][eo], (double)ke);
                        atomicAdd(&acc.abs_n[0][eo], 1u);
                    }
                    if (ci < 0 || ci >= N) {
                        want_i = false;
                        const int eo = ci < 0 ? 0 : 1;
                        atomicAdd(&acc.absK[1][eo], (double)ki);
                        atomicAdd(&acc.abs_n[1][eo], 1u);
                    }
                }
            }
        }
        const long long se = reserve_slot(want_e, gp(&st->n_child[0]), ns0, cap0);
        const long long si = reserve_slot(want_i, gp(&st->n_child[1]), ns1, cap1);
        if (want_e) {
            if (se >= 0) {
                // first trial of a child at the next step: draw 4 of its stream
                const uint4 r4 = philox((uint32_t)ch.ide, (uint32_t)(ch.ide >> 32), step32,
                                        4u, k0, k1);
                write_particle(C->sp[0], se, ce, oe, ch.vx, ch.vy, ch.vz, ch.ide,
                               wait_encode(geo0(r4.x, S.inv_log1mp)), kImp);
                deposit_global(C, 0, ce, oe);
            } else {
                atomicAdd(&acc.n_lost[0], 1u);
            }
        }
        if (want_i) {
            if (si >= 0) {
                const uint4 r4 = philox((uint32_t)ch.idi, (uint32_t)(ch.idi >> 32), step32,
                                        (1u << 28) | 4u, k0, k1);
                write_particle(C->sp[1], si, ci, oi, ch.ix, ch.iy, ch.iz, ch.idi,
                               wait_encode(geo0(r4.x, inv_ion)), kImp);
                deposit_global(C, 1, ci, oi);
            } else {
                atomicAdd(&acc.n_lost[1], 1u);
            }
        }
    };

    // the rounds of a list take its blocks of kBlock candidates in turn
    // (loading several candidates per thread ahead of their processing
    // measured slower: the loads are scattered, not latency-bound)
    for (int e0 = cw.round * kBlock; e0 < ncand; e0 += cw.rounds * kBlock) {
        const int e = e0 + tid;
        const bool act = e < ncand;
        int i = 0, c1 = 0;
        float o1 = 0.0f, vn = 0.0f, vn0 = 0.0f, abn = 0.0f, vy = 0.0f, vz = 0.0f;
        uint64_t id = 0;
        bool pred = false;  // implicit: k_step deposited the null prediction
        uint32_t nw = 0u;   // the particle's next waiting-time word
        int kind = -1;
        Child ch;
        if (act) {
            const uint32_t q4 = (uint32_t)(region + e) << 2;
            i = ldg(cq_idx, q4);
            vn = ldg(cq_vn, q4);
            if (kImp) abn = ldg(cq_ab, q4);
            const uint32_t i4 = (uint32_t)i << 2;
            // the list carries x_{n+1}; one 16-byte record holds id, vy, vz
            const int32_t w1 = ldg(cq_w, q4);
            if (kImp) o1 = ldg(cq_o, q4);
            const u32x4 r = ldg((const PIC_GLOBAL u32x4*)recp, i4 << 2);
            id = rec_id(r);
            vy = rec_vy(r);
            vz = rec_vz(r);
            c1 = cell_of(w1);
            vn0 = vn;
            pred = kImp && (wait_of(w1) & kPredDeposited);
            const float v2b = vn * vn + vy * vy + vz * vz;
            bool is_cand = true;
            if (wait_of(w1) & PIC_WAIT_CAPPED) {
                // a capped wait ran out: the trial of this step is drawn afresh
                const uint4 r4 = philox((uint32_t)id, (uint32_t)(id >> 32), step32,
                                        ((uint32_t)s << 28) | 4u, k0, k1);
                const double W = geo0(r4.x, S.inv_log1mp);
                if (W >= 1.0) {
                    is_cand = false;
                    nw = wait_encode(W - 1.0);
                }
            }
            if (is_cand) {
                const uint4 r0 = philox((uint32_t)id, (uint32_t)(id >> 32), step32,
                                        (uint32_t)s << 28, k0, k1);
                ++cand;
                nw = wait_encode(geo0(r0.x, S.inv_log1mp));
                bool over = false;
                kind = s == 0 ? collide_electron(S, lbound, r0, id, step32, k0, k1, vn, vy, vz,
                                                 over, ch)
                              : collide_ion(S, r0, id, step32, k0, k1, vn, vy, vz, over);
                if (over) atomicAdd(&acc.n_over, 1u);
            }
            if (kind >= 0) {
                atomicAdd(&acc.n_coll[kind], 1u);
                cdk += (double)(vn * vn + vy * vy + vz * vz - v2b);
                // vy, vz: the upper half of the record
                u32x2 yz;
                yz.x = __float_as_uint(vy);
                yz.y = __float_as_uint(vz);
                stg((PIC_GLOBAL u32x2*)recp, (i4 << 2) + 8u, yz);
            }
            if (DIAG && s == 0) {
                const float fb = (vn * vn + vy * vy + vz * vz) * eedf_k;
                const int bin = fb >= 1.0f ? min((int)fminf(fb, (float)kEedfBins), kEedfBins - 1) : 0;
                atomicAdd(&eedf[bin], 1u);
            }
        }
        // implicit: predict from the post-collision velocity, absorb, deposit
        bool dep_ok = false;
        int c2 = c1;
        float o2 = o1;
        if (act) {
            const uint32_t i4 = (uint32_t)i << 2;
            if (kImp && pred && kind < 0) {
                // a null collision: the prediction k_step stored and
                // deposited stands; only the waiting time is new
                predict(c2, o2, vn, abn);
                if (periodic) {
                    c2 %= N;
                    if (c2 < 0) c2 += N;
                }
                stg(cellp, i4, pack_cell(c2, nw));
            } else if (kImp) {
                if (pred) {
                    // a real collision: undo k_step's deposit of the null
                    // prediction (integer words, so exactly)
                    int cp = c1;
                    float op = o1;
                    predict(cp, op, vn0, abn);
                    if (periodic) {
                        cp %= N;
                        if (cp < 0) cp += N;
                    }
                    gatomic_add(&gdep_cnt[cp], ~0ull);
                    gatomic_add(&gdep_w[cp], 0ull - (packw(op) & kWMask));
                }
                const float vst = predict(c2, o2, vn, abn);
                bool gone = false;
                if (periodic) {
                    c2 %= N;
                    if (c2 < 0) c2 += N;
                } else if (c2 < 0 || c2 >= N) {
                    absorb(i, c2 < 0 ? 0 : 1, vn, vy, vz);
                    gone = true;
                }
                if (!gone) {
                    stg(cellp, i4, pack_cell(c2, nw));
                    stg(offp, i4, o2);
                    stg(vxp, i4, vst);
                    stg(abp, i4, abn);
                    dep_ok = true;
                }
            } else {
                if (kind >= 0) stg(vxp, i4, vn);   // the pass stored v_{n+1/2}
                stg(cellp, i4, pack_cell(c1, nw));
            }
        }
        if (kImp) deposit_wave(dep, dep_ok, c2, o2, lo, hi);
        // ionization children: queued in LDS and written after the loop, so
        // that a workgroup pays the latency of the slot reservation once;
        // events beyond the queue are handled here
        const bool ion_ev = act && kind == PIC_IONIZATION && s == 0;
        const unsigned long long im = __ballot(ion_ev);
        if (im) {
            const int leader = __ffsll((long long)im) - 1;
            int qb = 0;
            if (lane == leader) qb = atomicAdd(&q_n, (int)__popcll(im));
            qb = __shfl(qb, leader, 64);
            const int pos = qb + __popcll(im & ((1ull << lane) - 1ull));
            const bool queued = ion_ev && pos < kChildQ;
            if (queued) {
                ChildEv& q = cq[pos];
                q.parent = i;
                q.cell = c1;
                q.off = o1;
                q.ch = ch;
            }
            const bool now = ion_ev && !queued;
            if (__ballot(now)) {
                // explicit lists carry no offset: read it for the rare ionizations
                if (!kImp && now) o1 = ldg(offp, (uint32_t)i << 2);
                emit_children(now, c1, o1, ch);
            }
        }
    }
    // the queued ionizations: one event per thread
    lds_barrier();
    {
        const int nq = min(q_n, kChildQ);
        const bool ev = tid < nq;
        int c1 = 0;
        float o1 = 0.0f;
        Child ch{};
        if (ev) {
            const ChildEv& q = cq[tid];
            c1 = q.cell;
            o1 = kImp ? q.off : ldg(offp, (uint32_t)q.parent << 2);
            ch = q.ch;
        }
        if (__ballot(ev)) emit_children(ev, c1, o1, ch);
    }

    // flush the deposit of the implicit candidates and the EEDF counts
    if (kImp && hi >= 0) {
        atomicMin(&acc.cmin, lo);
        atomicMax(&acc.cmax, hi);
    }
    lds_barrier();
    if (kImp) {
        PIC_GLOBAL unsigned long long* gcnt = gp(C->dep_cnt[s]);
        PIC_GLOBAL unsigned long long* gw = gp(C->dep_w[s]);
        const int cl = acc.cmin, chh = acc.cmax;
        for (int j = cl + tid; chh >= 0 && j <= chh; j += kBlock) {
            const unsigned long long p = dep[j];
            if (p) {
                gatomic_add(&gcnt[j], p >> 40);
                gatomic_add(&gw[j], p & kWMask);
            }
        }
    }
    if (DIAG && s == 0)
        for (int j = tid; j < kEedfBins; j += kBlock)
            if (eedf[j]) gatomic_add(gp(&C->eedf_acc[j]), (unsigned long long)eedf[j]);
    // collision terms added to the workgroup's ledger row
    __shared__ double wsum[kWaves][2];
    cdk = wave_sum(cdk);
    const unsigned ncw = wave_sum(cand);
    if (lane == 0) {
        wsum[wave][0] = cdk;
        wsum[wave][1] = (double)ncw;
    }
    lds_barrier();
    // added to the row of the k_step workgroup whose list this is (its
    // collision fields start at zero; several rounds add in any order), one
    // field per thread
    if (tid < PD_N + PU_N) {
        const int o = 1 - s;
        const size_t S_ = (size_t)P.stride;
        if (tid < PD_N) {
            double x = 0.0;
            if (tid == PD_COLL + s)
                for (int k = 0; k < kWaves; ++k) x += wsum[k][0];
            else if (tid == PD_COLL + o && s == 0)
                x = acc.other_dK;
            else if (tid >= PD_ABSK && tid < PD_ABSK + 4)
                x = acc.absK[(tid - PD_ABSK) >> 1][(tid - PD_ABSK) & 1];
            if (x != 0.0) gatomic_add(gp(P.pd + (size_t)tid * S_ + gblk), x);
        } else {
            const int f = tid - PD_N;
            unsigned x = 0u;
            if (f >= PU_ABS && f < PU_ABS + 4) {
                x = acc.abs_n[(f - PU_ABS) >> 1][(f - PU_ABS) & 1];
            } else if (f >= PU_COLL + 4 * s && f < PU_COLL + 4 * s + 4) {
                x = acc.n_coll[f - PU_COLL - 4 * s];
            } else if (f == PU_CAND + s) {
                double nc = 0.0;
                for (int k = 0; k < kWaves; ++k) nc += wsum[k][1];
                x = (unsigned)nc;
            } else if (f == PU_CREATED + 0 || f == PU_CREATED + 1) {
                x = acc.n_created[f - PU_CREATED];
            } else if (f == PU_OVER + s) {
                x = acc.n_over;
            } else if (f == PU_LOST + 0 || f == PU_LOST + 1) {
                x = acc.n_lost[f - PU_LOST];
            }
            if (x != 0u) gatomic_add(gp(P.pu + (size_t)f * S_ + gblk), x);
        }
    }
}

// ---------------------------------------------------------------------------
// k_finalize: two workgroups per case after the particle pass, running side
// by side: the odd one closes the ledger of the step (reduction of the
// workgroup partials), the even one solves the FP64 field of the next step.
// They write disjoint fields of the case state (flags through atomics).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kFinBlock) void k_finalize(Params P, int sample)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kFinBlock / 64];
    __shared__ double sd[PD_N];
    __shared__ long long si[PU_N];
    Case* C = P.cases + (blockIdx.x >> 1);
    State* st = P.state + (blockIdx.x >> 1);
    if (blockIdx.x & 1) {
        // ledger of the step just taken
        reduce_partials<kFinBlock>(P.pd, P.pu, P.stride, C->first_block, C->n_blocks, sd, si);
        finish_ledger(C, st, sd, si);
        return;
    }
    // field of the next step (thread 0 alone reads and writes st->step)
    __shared__ long long s_step;
    if (threadIdx.x == 0) s_step = st->step;
    lds_barrier();
    const long long next = s_step + 1;
    solve_case<kFinBlock>(C, st, next + (C->scheme == 1 ? 1 : 0), next, sample != 0,
                          (double*)smem, red);
    if (threadIdx.x == 0) {
        if (sample) st->eedf_samples += 1;
        st->step = next;
    }
}

template __global__ void k_step<0, false>(Params);
template __global__ void k_step<0, true>(Params);
template __global__ void k_step<1, false>(Params);
template __global__ void k_step<1, true>(Params);
template __global__ void k_collide<0, false>(Params);
template __global__ void k_collide<0, true>(Params);
template __global__ void k_collide<1, false>(Params);
template __global__ void k_collide<1, true>(Params);

// ---------------------------------------------------------------------------
// Set-up: velocities from m/s to cells/step (unless given in internal
// units) and the D1 start-up prediction x~_1 = x_0 + v_{-1/2} dt.
// mode bit 0: convert units, bit 1: implicit start-up.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_init_species(Params P, double vscale0, double vscale1)
{
    const Work w = P.work[blockIdx.x];
    Case* C = P.cases + w.c;
    State* st = P.state + w.c;
    const Species& S = C->sp[w.s];
    const int N = C->n_cells;
    const int n = st->n_slots[w.s];
    int chunk = (n + w.nb - 1) / w.nb;
    chunk = (chunk + 63) & ~63;
    const int start = w.b * chunk, end = min(n, start + chunk);
    const double vs = w.s == 0 ? vscale0 : vscale1;
    const bool convert = P.mode & 1;
    const bool startup = (P.mode & 2) && C->scheme == 1;
    // waits drawn for a first trial at the start step (species loaded
    // without them, collisions on)
    const bool draw = ((P.mode >> (3 + w.s)) & 1) && C->collisions && S.n_proc > 0;
    const uint32_t step32 = (uint32_t)st->step;
    for (int i = start + (int)threadIdx.x; i < end; i += kBlock) {
        if (convert) {
            S.vx[i] = (float)((double)S.vx[i] * vs);
            const u32x4 r = S.rec[i];
            S.rec[i] = make_rec(rec_id(r), (float)((double)rec_vy(r) * vs),
                                (float)((double)rec_vz(r) * vs));
        }
        const int32_t word = S.cell[i];
        if (word < 0) continue;
        int c = cell_of(word);
        uint32_t wt = wait_of(word);
        if (draw) {
            const uint64_t id = rec_id(S.rec[i]);
            const uint4 r4 = philox((uint32_t)id, (uint32_t)(id >> 32), step32,
                                    ((uint32_t)w.s << 28) | 4u, C->key0, C->key1);
            wt = wait_encode(geo0(r4.x, S.inv_log1mp));
        }
        float o = S.off[i];
        if (startup) {
            S.abar[i] = 0.0f;
            o += S.vx[i];
            renorm(c, o);
            if (C->bc == 1) {
                c %= N;
                if (c < 0) c += N;
            } else if (c < 0 || c >= N) {
                S.cell[i] = -1;
                continue;
            }
            S.off[i] = o;
        }
        S.cell[i] = pack_cell(c, wt);
    }
}

// LDS counter increment for the valid lanes of a wavefront.  Returns, for
// each valid lane, the value a plain atomicAdd of 1 would have returned (its
// slot).  When all valid lanes hit one cell (cell-sorted particles) a single
// atomic serves the wavefront.
__device__ __forceinline__ unsigned wave_count_add(unsigned* h, int c, bool valid)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long m = __ballot(valid);
    if (m == 0ull) return 0u;
    const int leader = __ffsll((long long)m) - 1;
    const int key = __shfl(c, leader, 64);
    if (__ballot(valid && c != key) == 0ull) {
        // every valid lane hits one cell: one atomic for the wavefront
        unsigned base = 0u;
        if (lane == leader) base = atomicAdd(&h[key], (unsigned)__popcll(m));
        base = __shfl(base, leader, 64);
        return base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
    }
    return valid ? atomicAdd(&h[c], 1u) : 0u;
}

// ---------------------------------------------------------------------------
// Compaction: drop absorbed slots and sort every species by bucket with a
// counting sort across workgroups (the order inside one bucket is
// arbitrary).  Ions are sorted by cell; electrons, which cross many cells
// between sorts, by buckets of 2^kElecBucketShift cells, so that every
// workgroup writes its particles in a few long runs (the writes of a run
// complete cache lines while they are resident instead of trickling out as
// partial lines).
// ---------------------------------------------------------------------------
constexpr int kElecBucketShift = 4;

__device__ __forceinline__ int bucket_shift(int s) { return s == 0 ? kElecBucketShift : 0; }
__device__ __forceinline__ int n_buckets(int N, int s)
{
    return (N + (1 << bucket_shift(s)) - 1) >> bucket_shift(s);
}

__global__ __launch_bounds__(kBlock) void k_compact_hist(Params P, uint32_t* hist_all,
                                                         const int64_t* hist_off)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_lo, s_hi;
    const Work w = P.work[blockIdx.x];
    Case* C = P.cases + w.c;
    State* st = P.state + w.c;
    const int sh = bucket_shift(w.s);
    const int NB = n_buckets(C->n_cells, w.s);
    const PIC_GLOBAL int32_t* __restrict__ cellp = gp((const int32_t*)C->sp[w.s].cell);
    PIC_GLOBAL uint32_t* hist = gp(hist_all + hist_off[2 * w.c + w.s]);
    unsigned* lh = (unsigned*)smem;
    for (int j = threadIdx.x; j < NB; j += kBlock) lh[j] = 0u;
    if (threadIdx.x == 0) {
        s_lo = kNoCell;
        s_hi = -1;
    }
    lds_barrier();
    const int n = st->n_slots[w.s];
    int chunk = (n + w.nb - 1) / w.nb;
    chunk = (chunk + 63) & ~63;
    const int start = w.b * chunk, end = min(n, start + chunk);
    int lo = kNoCell, hi = -1;
    for (int base = start; base < end; base += kBlock) {
        const int i = base + (int)threadIdx.x;
        const int c = i < end ? cell_of(cellp[i]) : -1;
        const int b = c >= 0 ? c >> sh : -1;
        wave_count_add(lh, b, b >= 0);
        if (b >= 0) range_note(lo, hi, b);
    }
    if (hi >= 0) {
        atomicMin(&s_lo, lo);
        atomicMax(&s_hi, hi);
    }
    lds_barrier();
    for (int j = s_lo + (int)threadIdx.x; s_hi >= 0 && j <= s_hi; j += kBlock)
        if (lh[j]) gatomic_add(&hist[j], lh[j]);
}

// one workgroup per (case, species): exclusive scan of the histogram
__global__ __launch_bounds__(kBlock) void k_compact_scan(Params P, uint32_t* hist_all,
                                                         uint32_t* cursor_all,
                                                         const int64_t* hist_off)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned red[kWaves];
    const int c = blockIdx.x >> 1, s = blockIdx.x & 1;
    Case* C = P.cases + c;
    State* st = P.state + c;
    const int NB = n_buckets(C->n_cells, s);
    PIC_GLOBAL uint32_t* hist = gp(hist_all + hist_off[2 * c + s]);
    PIC_GLOBAL uint32_t* cur = gp(cursor_all + hist_off[2 * c + s]);
    unsigned* a = (unsigned*)smem;
    for (int j = threadIdx.x; j < NB; j += kBlock) {
        a[j] = hist[j];
        hist[j] = 0u;
    }
    lds_barrier();
    block_scan(a, NB, red);
    for (int j = threadIdx.x; j < NB; j += kBlock) cur[j] = j > 0 ? a[j - 1] : 0u;
    if (threadIdx.x == 0) st->sort_live[s] = NB > 0 ? a[NB - 1] : 0;
}

__global__ __launch_bounds__(kBlock) void k_compact_scatter(Params P, uint32_t* cursor_all,
                                                            const int64_t* hist_off)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_lo, s_hi;
    __shared__ double red[kWaves];
    const Work w = P.work[blockIdx.x];
    Case* C = P.cases + w.c;
    State* st = P.state + w.c;
    const Species S = C->sp[w.s];
    const int sh = bucket_shift(w.s);
    const int NB = n_buckets(C->n_cells, w.s);
    const bool imp = C->scheme == 1;
    PIC_GLOBAL uint32_t* cur = gp(cursor_all + hist_off[2 * w.c + w.s]);
    unsigned* lh = (unsigned*)smem;
    unsigned* lb = lh + NB;
    for (int j = threadIdx.x; j < NB; j += kBlock) lh[j] = 0u;
    if (threadIdx.x == 0) {
        s_lo = kNoCell;
        s_hi = -1;
    }
    lds_barrier();
    const int n = st->n_slots[w.s];
    int chunk = (n + w.nb - 1) / w.nb;
    chunk = (chunk + 63) & ~63;
    const int start = w.b * chunk, end = min(n, start + chunk);
    const PIC_GLOBAL int32_t* __restrict__ cellp = gp((const int32_t*)S.cell);
    int lo = kNoCell, hi = -1;
    for (int base = start; base < end; base += kBlock) {
        const int i = base + (int)threadIdx.x;
        const int c = i < end ? cell_of(cellp[i]) : -1;
        const int b = c >= 0 ? c >> sh : -1;
        wave_count_add(lh, b, b >= 0);
        if (b >= 0) range_note(lo, hi, b);
    }
    if (hi >= 0) {
        atomicMin(&s_lo, lo);
        atomicMax(&s_hi, hi);
    }
    lds_barrier();
    // one run per touched bucket
    for (int j = s_lo + (int)threadIdx.x; s_hi >= 0 && j <= s_hi; j += kBlock) {
        const unsigned k = lh[j];
        if (k) lb[j] = gatomic_add(&cur[j], k);
        lh[j] = 0u;
    }
    lds_barrier();
    const PIC_GLOBAL float* __restrict__ offp = gp((const float*)S.off);
    const PIC_GLOBAL float* __restrict__ vxp = gp((const float*)S.vx);
    const PIC_GLOBAL u32x4* __restrict__ recp = gp((const u32x4*)S.rec);
    const PIC_GLOBAL float* __restrict__ abp = gp((const float*)S.abar);
    PIC_GLOBAL int32_t* __restrict__ cell2 = gp(S.cell2);
    PIC_GLOBAL float* __restrict__ off2 = gp(S.off2);
    PIC_GLOBAL float* __restrict__ vx2 = gp(S.vx2);
    PIC_GLOBAL u32x4* __restrict__ rec2 = gp(S.rec2);
    PIC_GLOBAL float* __restrict__ ab2 = gp(S.abar2);
    double v2 = 0.0;
    for (int base = start; base < end; base += kBlock) {
        const int i = base + (int)threadIdx.x;
        const int j = min(i, end - 1);
        const int32_t w0 = cellp[j];
        const float o = offp[j], vx = vxp[j];
        const u32x4 rc = recp[j];
        const float vy = rec_vy(rc), vz = rec_vz(rc);
        const float ab = imp ? abp[j] : 0.0f;
        const int c = i < end ? cell_of(w0) : -1;
        const int b = c >= 0 ? c >> sh : -1;
        const unsigned r = wave_count_add(lh, b, b >= 0);
        if (c < 0) continue;
        const unsigned d = lb[b] + r;
        cell2[d] = w0;
        off2[d] = o;
        vx2[d] = vx;
        rec2[d] = rc;
        float vh = vx;
        if (imp) {
            ab2[d] = ab;
            vh = vx - 0.5f * ab;   // v_{n-1/2} from the stored prediction
        }
        v2 += (double)(vh * vh + vy * vy + vz * vz);
    }
    v2 = block_sum(v2, red);
    if (threadIdx.x == 0) {
        P.pd[(size_t)(PD_V2 + w.s) * P.stride + blockIdx.x] = v2;
        P.pd[(size_t)(PD_V2 + 1 - w.s) * P.stride + blockIdx.x] = 0.0;
    }
}

// one workgroup per case: swap buffers, set counts and the exact kinetic energy
__global__ __launch_bounds__(kFinBlock) void k_compact_finish(Params P)
{
    __shared__ double sd[PD_N];
    __shared__ long long si[PU_N];
    Case* C = P.cases + blockIdx.x;
    State* st = P.state + blockIdx.x;
    reduce_partials<kFinBlock>(P.pd, P.pu, P.stride, C->first_block, C->n_blocks, sd, si);
    if (threadIdx.x != 0) return;
    for (int s = 0; s < 2; ++s) {
        Species& S = C->sp[s];
        st->K[s] = sd[PD_V2 + s] * S.kin_unit;
        st->sortK[s] = st->K[s];
        const int live = (int)st->sort_live[s];
        st->n_slots[s] = live;
        st->n_live[s] = live;
        int32_t* t0 = S.cell; S.cell = S.cell2; S.cell2 = t0;
        float* t1 = S.off; S.off = S.off2; S.off2 = t1;
        t1 = S.vx; S.vx = S.vx2; S.vx2 = t1;
        u32x4* t2 = S.rec; S.rec = S.rec2; S.rec2 = t2;
        t1 = S.abar; S.abar = S.abar2; S.abar2 = t1;
    }
}

// Deposit of the stored positions (set-up), then k_solve per case.
__global__ __launch_bounds__(kBlock) void k_deposit(Params P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_lo, s_hi;
    const Work w = P.work[blockIdx.x];
    Case* C = P.cases + w.c;
    State* st = P.state + w.c;
    const Species& S = C->sp[w.s];
    const int N = C->n_cells;
    unsigned long long* dep = (unsigned long long*)smem;
    for (int j = threadIdx.x; j <= N; j += kBlock) dep[j] = 0ull;
    const bool ec2 = C->gather == 2, periodic = C->bc == 1;
    if (threadIdx.x == 0) {
        s_lo = kNoCell;
        s_hi = -1;
    }
    lds_barrier();
    const int n = st->n_slots[w.s];
    int chunk = (n + w.nb - 1) / w.nb;
    chunk = (chunk + 63) & ~63;
    const int start = w.b * chunk, end = min(n, start + chunk);
    int lo = kNoCell, hi = -1;
    for (int i = start + (int)threadIdx.x; i < end; i += kBlock) {
        const int c = cell_of(S.cell[i]);
        if (c < 0) continue;
        if (ec2) {
            deposit_quad(dep, true, c, S.off[i], N, periodic, lo, hi);
        } else {
            atomicAdd(&dep[c], packw(S.off[i]));
            range_note(lo, hi, c);
        }
    }
    if (hi >= 0) {
        atomicMin(&s_lo, lo);
        atomicMax(&s_hi, hi);
    }
    lds_barrier();
    for (int j = s_lo + (int)threadIdx.x; s_hi >= 0 && j <= s_hi; j += kBlock) {
        const unsigned long long p = dep[j];
        if (p) {
            atomicAdd(&C->dep_cnt[w.s][j], p >> 40);
            atomicAdd(&C->dep_w[w.s][j], p & kWMask);
        }
    }
}

__global__ __launch_bounds__(kFinBlock) void k_solve(Params P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kFinBlock / 64];
    Case* C = P.cases + blockIdx.x;
    State* st = P.state + blockIdx.x;
    solve_case<kFinBlock>(C, st, st->step + (C->scheme == 1 ? 1 : 0), st->step, false,
                          (double*)smem, red);
}

}  // namespace pic
