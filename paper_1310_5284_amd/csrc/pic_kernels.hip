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

__device__ void solve_case(Case* C, State* st, long long next_step, bool sample_density,
                           double* S, double* red)
{
    const int N = C->n_cells, tid = threadIdx.x;
    const bool periodic = C->bc == 1;
    const bool implicit = C->scheme == 1;
    const double dx = C->dx;
    // node charges from the per-cell counts and weights
    for (int g = tid; g <= N; g += kBlock) {
        double rho = C->background_rho;
        const int gg = (periodic && g == N) ? 0 : g;
        for (int s = 0; s < 2; ++s) {
            const long long cg = gg < N ? (long long)C->dep_cnt[s][gg] : 0;
            const long long wg = gg < N ? (long long)C->dep_w[s][gg] : 0;
            long long wl = 0;
            if (gg > 0) wl = (long long)C->dep_w[s][gg - 1];
            else if (periodic) wl = (long long)C->dep_w[s][N - 1];
            const long long q = cg * (1ll << kFixBits) - wg + wl;
            C->qfix[s][g] = q;
            if (sample_density) atomicAdd(&C->dens_acc[s][g], (unsigned long long)q);
            rho += (double)q * (C->sp[s].qw_dx / kFixScale);
        }
        C->rho[g] = rho;
        S[g] = rho;
    }
    for (int j = tid; j < N; j += kBlock) {
        const long long ce = (long long)C->dep_cnt[0][j], ci = (long long)C->dep_cnt[1][j];
        C->ccount[0][j] = ce;
        C->ccount[1][j] = ci;
        C->chi[j] = implicit ? C->sp[0].chi_coef * (double)ce + C->sp[1].chi_coef * (double)ci
                             : 0.0;
    }
    __syncthreads();
    for (int j = tid; j < N; j += kBlock) {
        C->dep_cnt[0][j] = 0; C->dep_cnt[1][j] = 0;
        C->dep_w[0][j] = 0; C->dep_w[1][j] = 0;
    }
    if (tid == 0) S[0] = 0.0;
    __syncthreads();
    for (int k = 1 + tid; k < N; k += kBlock) S[k] *= dx;
    __syncthreads();
    block_scan(S, N, red);                          // S[j] = R_j
    double a = 0.0, b = 0.0;
    for (int j = tid; j < N; j += kBlock) {
        const double kap = kEps0 * (1.0 + C->chi[j]);
        a += S[j] / kap;
        b += 1.0 / kap;
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    double V = 0.0;
    if (!periodic) V = C->rf_volts * sin(C->rf_omega * ((double)next_step * C->dt));
    const double D0 = (V / dx - a) / b;
    double we = 0.0;
    for (int j = tid; j < N; j += kBlock) {
        const double kap = kEps0 * (1.0 + C->chi[j]);
        const double E = (D0 + S[j]) / kap;
        C->E[j] = E;
        C->ehat[0][j] = (float)(C->sp[0].accel * E);
        C->ehat[1][j] = (float)(C->sp[1].accel * E);
        we += 0.5 * kEps0 * E * E * dx;
    }
    __syncthreads();
    for (int j = tid; j < N; j += kBlock) S[j] = C->E[j];
    we = block_sum(we, red);
    block_scan(S, N, red);
    const double phi0 = periodic ? 0.0 : V;
    if (tid == 0) C->phi[0] = phi0;
    for (int j = tid; j < N; j += kBlock) C->phi[j + 1] = phi0 - dx * S[j];
    if (tid == 0) {
        st->WE = we;
        if (!isfinite(we)) st->flags |= 1;
        if (sample_density) st->dens_samples += 1;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Ledger: the finalizing workgroup reduces the per-workgroup partials of its
// case in a fixed order and appends one row.
// ---------------------------------------------------------------------------
__device__ void finish_ledger(Case* C, State* st, const Partial* parts, double* red)
{
    const int tid = threadIdx.x;
    const int nb = C->n_blocks, fb = C->first_block;
    constexpr int kD = 10, kI = 20;
    __shared__ double sd[kD];
    __shared__ long long si[kI];
    for (int f = 0; f < kD; ++f) {
        double v = 0.0;
        for (int b = tid; b < nb; b += kBlock) v += (&parts[fb + b].work[0])[f];
        v = block_sum(v, red);
        if (tid == 0) sd[f] = v;
    }
    for (int f = 0; f < kI; ++f) {
        long long v = 0;
        for (int b = tid; b < nb; b += kBlock) v += (&parts[fb + b].abs_n[0][0])[f];
        v = block_sum(v, (long long*)red);
        if (tid == 0) si[f] = v;
    }
    __syncthreads();
    if (tid != 0) return;
    // field order of Partial: work[2], coll_dK[2], absK[2][2], v2sum[2]; then
    // abs_n[2][2], n_coll[2][4], n_cand[2], n_created[2], n_over[2], n_lost[2]
    pic_ledger L;
    L.step = st->step;
    L.WE = st->WE;
    for (int s = 0; s < 2; ++s) {
        const double ku = C->sp[s].kin_unit;
        L.K_before[s] = st->K[s];
        L.work[s] = sd[0 + s] * ku;
        L.coll_dK[s] = sd[2 + s] * ku;
        L.absorbed_K[s][0] = sd[4 + 2 * s] * ku;
        L.absorbed_K[s][1] = sd[5 + 2 * s] * ku;
        L.K_after[s] = L.K_before[s] + L.work[s] - L.absorbed_K[s][0] - L.absorbed_K[s][1] +
                       L.coll_dK[s];
        st->K[s] = L.K_after[s];
        L.absorbed_n[s][0] = si[0 + 2 * s];
        L.absorbed_n[s][1] = si[1 + 2 * s];
        for (int k = 0; k < 4; ++k) L.n_coll[s][k] = si[4 + 4 * s + k];
        L.n_candidates[s] = si[12 + s];
        L.n_created[s] = si[14 + s];
        L.n_over_table[s] = si[16 + s];
        L.n_lost[s] = si[18 + s];
        st->n_live[s] += (int32_t)(L.n_created[s] - L.absorbed_n[s][0] - L.absorbed_n[s][1]);
        st->lost_total[s] += L.n_lost[s];
        const long long ns = (long long)st->n_slots[s] + st->n_child[s];
        const long long cap = C->sp[s].capacity;
        st->n_slots[s] = (int32_t)(ns < cap ? ns : cap);
        if (ns > cap || L.n_lost[s] > 0) st->flags |= 2;
        st->n_child[s] = 0;
    }
    if (!isfinite(L.K_after[0]) || !isfinite(L.K_after[1])) st->flags |= 1;
    pic_ledger* H = (pic_ledger*)C->history;
    H[0] = L;
    if (C->history_len > 0) H[1 + (st->history_n % C->history_len)] = L;
    st->history_n += 1;
}

// ---------------------------------------------------------------------------
// Shared-memory layout of k_step: ehat[N] float | dep[N] u64 | (DIAG) heat[N]
// float | eedf[kEedfBins] u32.  The finalizer reuses it as N+1 doubles.
// ---------------------------------------------------------------------------
__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

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

// MC gather: CIC of the nodal field E_g = (E_{g-1/2} + E_{g+1/2}) / 2
__device__ __forceinline__ float gather_mc(const float* eh, int N, bool periodic, int c, float o)
{
    auto node = [&](int g) -> float {
        if (periodic) {
            const int gl = g == 0 ? N - 1 : g - 1;
            const int gr = g == N ? 0 : g;
            return 0.5f * (eh[gl] + eh[gr]);
        }
        if (g == 0) return eh[0];
        if (g == N) return eh[N - 1];
        return 0.5f * (eh[g - 1] + eh[g]);
    };
    return (1.0f - o) * node(c) + o * node(c + 1);
}

__device__ __forceinline__ unsigned long long packw(float o)
{
    return kCountOne + (unsigned long long)__float2uint_rn(o * 16777216.0f);
}

// ---------------------------------------------------------------------------
// Collision of one candidate (null-collision MCC, Vahedi & Surendra 1995).
// Returns the process kind or -2 (null).  Velocities in cells/step.
// ---------------------------------------------------------------------------
struct Child {
    float vx, vy, vz;
    float ix, iy, iz;   // new ion
    uint64_t ide, idi;
};

__device__ __forceinline__ int collide_electron(const Species& S, uint4 r0, uint64_t id,
                                                uint32_t step, uint32_t k0, uint32_t k1,
                                                float& vx, float& vy, float& vz, bool& over,
                                                Child& ch)
{
    const float v2 = vx * vx + vy * vy + vz * vz;
    const float vm = sqrtf(v2);
    const float t = fmaf(v2, S.t_scale, S.t_off);
    over = t > S.t_max;
    const float tc = fminf(fmaxf(t, 0.0f), S.t_max);
    const int k = min((int)tc, (int)S.t_max - 1);
    const float f = tc - (float)k;
    const float4 A = S.tab_e[k], B = S.tab_e[k + 1];
    float sg[4] = {fmaf(f, B.x - A.x, A.x), fmaf(f, B.y - A.y, A.y), fmaf(f, B.z - A.z, A.z),
                   fmaf(f, B.w - A.w, A.w)};
    const float u1 = u01(r0.y);
    int slot = -1;
    float cum = 0.0f;
#pragma unroll
    for (int p = 0; p < kMaxProc; ++p) {
        if (p < S.n_proc && slot < 0) {
            const float sp = v2 > S.thr_v2[p] ? sg[p] : 0.0f;
            cum += sp * vm;
            if (u1 < cum) slot = p;
        }
    }
    if (slot < 0) return -2;
    const int kind = S.kind[slot];
    float dx, dy, dz;
    iso_dir(u01(r0.z), u01(r0.w), dx, dy, dz);
    if (kind == PIC_ELASTIC) {
        const float cchi = vm > 0.0f ? (vx * dx + vy * dy + vz * dz) / vm : 0.0f;
        const float sp = sqrtf(v2 * (1.0f - S.recoil2 * (1.0f - cchi)));
        vx = sp * dx; vy = sp * dy; vz = sp * dz;
    } else if (kind == PIC_EXCITATION) {
        const float sp = sqrtf(fmaxf(v2 - S.thr_v2[slot], 0.0f));
        vx = sp * dx; vy = sp * dy; vz = sp * dz;
    } else if (kind == PIC_IONIZATION) {
        const uint4 r1 = philox((uint32_t)id, (uint32_t)(id >> 32), step, 1u, k0, k1);
        const uint4 r3 = philox((uint32_t)id, (uint32_t)(id >> 32), step, 3u, k0, k1);
        const float B = S.opal_B;
        const float avail = fmaxf(v2 - S.thr_v2[slot], 0.0f) * S.eps_unit;   // eV
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
    const float a = S.tab_i[k], b = S.tab_i[k + 1];
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
struct ChildSink {
    Case* C;
    State* st;
    int n_slots0, n_slots1;
};

// Reserve slots for the lanes with want = true; returns the slot or -1.
__device__ __forceinline__ long long reserve_slot(bool want, int32_t* counter, int base_slots,
                                                  long long cap)
{
    const unsigned long long m = __ballot(want);
    if (m == 0) return -1;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    int b = 0;
    if (lane == leader) b = atomicAdd(counter, __popcll(m));
    b = __shfl(b, leader, 64);
    if (!want) return -1;
    const long long slot = (long long)base_slots + b + rank;
    return slot < cap ? slot : -2;
}

__device__ __forceinline__ void write_particle(const Species& S, long long slot, int c, float o,
                                               float vx, float vy, float vz, uint64_t id,
                                               bool implicit)
{
    S.cell[slot] = c;
    S.off[slot] = o;
    S.vx[slot] = vx;
    S.vy[slot] = vy;
    S.vz[slot] = vz;
    S.id[slot] = id;
    if (implicit) S.abar[slot] = 0.0f;
}

// ---------------------------------------------------------------------------
// k_step: one step of every case in this launch.  Workgroup = a contiguous
// chunk of one species of one case.  Per particle (explicit, leap-frog):
//   a = ehat[cell] (EC, Eq. (3)) or CIC of the nodal field (MC);
//   v += a;  x += v;  absorb at the electrodes or wrap;
//   null-collision MCC with Philox(id, step);  deposit (Eq. (2)).
// Per particle (implicit, D1, beta = 1/2; stored x~, v~, abar):
//   a = ehat[cell of x~];  x = x~ + a/2;  v = v~ + a/2;  abar = (abar + a)/2;
//   absorb; MCC; predict v~' = v + abar/2, x~' = x + v~'; absorb; deposit x~'.
// The deposit goes to a privatised LDS copy of the grid (one int64 per cell
// packs count and summed weight) and is flushed over the cell range the
// workgroup touched.  The last workgroup of a case closes the ledger and
// solves the field of the next step.
// ---------------------------------------------------------------------------
template <int SCHEME, bool DIAG>
__global__ __launch_bounds__(kBlock) void k_step(Params P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ BlockAcc acc;
    __shared__ double red[kWaves];
    __shared__ int s_last;
    constexpr bool kImp = SCHEME == 1;
    const int tid = threadIdx.x;
    const int gblk = P.mode + (int)blockIdx.x;
    const Work w = P.work[gblk];
    Case* C = P.cases + w.c;
    State* st = P.state + w.c;
    const int N = C->n_cells;
    const int s = w.s;
    const Species& S = C->sp[s];
    const bool periodic = C->bc == 1;
    const bool mc = C->gather == 1;
    const bool coll = C->collisions != 0 && S.n_proc > 0;
    const uint32_t k0 = C->key0, k1 = C->key1;

    float* eh = (float*)smem;
    unsigned long long* dep = (unsigned long long*)(smem + align16(4 * (size_t)N));
    float* heat = (float*)(smem + align16(4 * (size_t)N) + align16(8 * (size_t)N));
    unsigned* eedf = (unsigned*)(smem + 2 * align16(4 * (size_t)N) + align16(8 * (size_t)N));

    for (int j = tid; j < N; j += kBlock) {
        eh[j] = C->ehat[s][j];
        dep[j] = 0ull;
        if (DIAG) heat[j] = 0.0f;
    }
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
    }
    __syncthreads();

    const uint32_t step32 = (uint32_t)st->step;
    const int n = st->n_slots[s];
    const int ns0 = st->n_slots[0], ns1 = st->n_slots[1];
    int chunk = (n + w.nb - 1) / w.nb;
    chunk = (chunk + 63) & ~63;
    const int start = w.b * chunk;
    const int end = min(n, start + chunk);

    int32_t* __restrict__ cellp = S.cell;
    float* __restrict__ offp = S.off;
    float* __restrict__ vxp = S.vx;
    float* __restrict__ vyp = S.vy;
    float* __restrict__ vzp = S.vz;
    const uint64_t* __restrict__ idp = S.id;
    float* __restrict__ abp = S.abar;

    double work = 0.0, cdk = 0.0;
    unsigned cand = 0u;
    int lo = kNoCell, hi = -1;

    for (int base = start; base < end; base += kBlock) {
        const int i = base + tid;
        const bool in = i < end;
        int c = in ? cellp[i] : -1;
        bool live = c >= 0;
        float o = 0.0f, v = 0.0f, ab = 0.0f, a = 0.0f;
        if (live) {
            o = offp[i];
            v = vxp[i];
            if (kImp) ab = abp[i];
            a = mc ? gather_mc(eh, N, periodic, c, o) : eh[c];
        }
        // push: vn is v_{n+1/2}; (c2, o2) the position the step ends at
        float vn, ab_n = 0.0f, vold;
        int c1 = c;
        float o1 = o;
        if (kImp) {
            vold = v - 0.5f * ab;
            vn = v + 0.5f * a;
            ab_n = 0.5f * (ab + a);
            o1 = o + 0.5f * a;
        } else {
            vold = v;
            vn = v + a;
            o1 = o + vn;
        }
        if (live) {
            const float dk = (vn - vold) * (vn + vold);
            work += (double)dk;
            if (DIAG) {
                atomicAdd(&heat[c], dk);
                range_note(lo, hi, c);
            }
            renorm(c1, o1);
        }
        float vy = 0.0f, vz = 0.0f;
        bool have_yz = false, dirty = false;
        // boundary at x_{n+1}
        if (live) {
            if (periodic) {
                c1 %= N;
                if (c1 < 0) c1 += N;
            } else if (c1 < 0 || c1 >= N) {
                vy = vyp[i];
                vz = vzp[i];
                const int e = c1 < 0 ? 0 : 1;
                atomicAdd(&acc.absK[s][e], (double)(vn * vn + vy * vy + vz * vz));
                atomicAdd(&acc.abs_n[s][e], 1u);
                cellp[i] = -1;
                live = false;
            }
        }
        int kind = -1;
        Child ch;
        uint64_t id = 0;
        if (live && coll) {
            id = idp[i];
            const uint4 r0 = philox((uint32_t)id, (uint32_t)(id >> 32), step32,
                                    (uint32_t)s << 28, k0, k1);
            if ((r0.x >> 9) < S.cand_thr) {
                ++cand;
                vy = vyp[i];
                vz = vzp[i];
                have_yz = true;
                const float v2b = vn * vn + vy * vy + vz * vz;
                bool over = false;
                kind = s == 0 ? collide_electron(S, r0, id, step32, k0, k1, vn, vy, vz, over, ch)
                              : collide_ion(S, r0, id, step32, k0, k1, vn, vy, vz, over);
                if (over) atomicAdd(&acc.n_over, 1u);
                if (kind >= 0) {
                    dirty = true;
                    atomicAdd(&acc.n_coll[kind], 1u);
                    cdk += (double)(vn * vn + vy * vy + vz * vz - v2b);
                }
            }
        }
        if (DIAG && s == 0 && live) {
            if (!have_yz) {
                vy = vyp[i];
                vz = vzp[i];
            }
            const float eps = (vn * vn + vy * vy + vz * vz) * S.eps_unit;
            const float fb = eps * S.eedf_scale;   // NaN or negative -> bin 0
            const int bin = fb >= 1.0f ? min((int)fminf(fb, (float)kEedfBins), kEedfBins - 1) : 0;
            atomicAdd(&eedf[bin], 1u);
        }
        // predicted position (implicit) or final position (explicit)
        int c2 = c1;
        float o2 = o1, vst = vn;
        if (kImp && live) {
            vst = vn + 0.5f * ab_n;
            o2 = o1 + vst;
            renorm(c2, o2);
            if (periodic) {
                c2 %= N;
                if (c2 < 0) c2 += N;
            } else if (c2 < 0 || c2 >= N) {
                if (!have_yz) {
                    vy = vyp[i];
                    vz = vzp[i];
                }
                const int e = c2 < 0 ? 0 : 1;
                atomicAdd(&acc.absK[s][e], (double)(vn * vn + vy * vy + vz * vz));
                atomicAdd(&acc.abs_n[s][e], 1u);
                cellp[i] = -1;
                live = false;
            }
        }
        if (live) {
            atomicAdd(&dep[c2], packw(o2));
            range_note(lo, hi, c2);
            cellp[i] = c2;
            offp[i] = o2;
            vxp[i] = vst;
            if (kImp) abp[i] = ab_n;
            if (dirty) {
                vyp[i] = vy;
                vzp[i] = vz;
            }
        }
        // ionization children: electron and ion at the parent's x_{n+1};
        // implicit children are predicted from there with abar = 0
        const bool ion_ev = kind == PIC_IONIZATION && s == 0;
        if (__ballot(ion_ev)) {
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
                            const int e = ce < 0 ? 0 : 1;
                            atomicAdd(&acc.absK[0][e], (double)ke);
                            atomicAdd(&acc.abs_n[0][e], 1u);
                        }
                        if (ci < 0 || ci >= N) {
                            want_i = false;
                            const int e = ci < 0 ? 0 : 1;
                            atomicAdd(&acc.absK[1][e], (double)ki);
                            atomicAdd(&acc.abs_n[1][e], 1u);
                        }
                    }
                }
            }
            const long long se = reserve_slot(want_e, &st->n_child[0], ns0, C->sp[0].capacity);
            const long long si = reserve_slot(want_i, &st->n_child[1], ns1, C->sp[1].capacity);
            if (want_e) {
                if (se >= 0) {
                    write_particle(C->sp[0], se, ce, oe, ch.vx, ch.vy, ch.vz, ch.ide, kImp);
                    atomicAdd(&dep[ce], packw(oe));
                    range_note(lo, hi, ce);
                } else {
                    atomicAdd(&acc.n_lost[0], 1u);
                }
            }
            if (want_i) {
                if (si >= 0) {
                    write_particle(C->sp[1], si, ci, oi, ch.ix, ch.iy, ch.iz, ch.idi, kImp);
                    atomicAdd(&C->dep_cnt[1][ci], 1ull);
                    atomicAdd(&C->dep_w[1][ci], packw(oi) & kWMask);
                } else {
                    atomicAdd(&acc.n_lost[1], 1u);
                }
            }
        }
    }

    // flush the privatised deposit over the touched cell range
    if (hi >= 0) {
        atomicMin(&acc.cmin, lo);
        atomicMax(&acc.cmax, hi);
    }
    __syncthreads();
    {
        const int cl = acc.cmin, chh = acc.cmax;
        for (int j = cl + tid; chh >= 0 && j <= chh; j += kBlock) {
            const unsigned long long p = dep[j];
            if (p) {
                atomicAdd(&C->dep_cnt[s][j], p >> 40);
                atomicAdd(&C->dep_w[s][j], p & kWMask);
            }
            if (DIAG) {
                const float h = heat[j];
                if (h != 0.0f) atomicAdd(&C->heat_acc[s][j], (double)h * S.kin_unit);
            }
        }
        if (DIAG && s == 0)
            for (int j = tid; j < kEedfBins; j += kBlock)
                if (eedf[j]) atomicAdd(&C->eedf_acc[j], (unsigned long long)eedf[j]);
    }
    // workgroup partial of the ledger
    work = block_sum(work, red);
    cdk = block_sum(cdk, red);
    const unsigned ncand = block_sum(cand, (unsigned*)red);
    if (tid == 0) {
        Partial& pp = P.partials[gblk];
        const int o = 1 - s;
        pp.work[s] = work;
        pp.work[o] = 0.0;
        pp.coll_dK[s] = cdk;
        pp.coll_dK[o] = s == 0 ? acc.other_dK : 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                pp.absK[a][b] = acc.absK[a][b];
                pp.abs_n[a][b] = acc.abs_n[a][b];
            }
        pp.v2sum[0] = pp.v2sum[1] = 0.0;
        for (int k = 0; k < 4; ++k) {
            pp.n_coll[s][k] = acc.n_coll[k];
            pp.n_coll[o][k] = 0;
        }
        pp.n_cand[s] = ncand;
        pp.n_cand[o] = 0;
        pp.n_created[0] = acc.n_created[0];
        pp.n_created[1] = acc.n_created[1];
        pp.n_over[s] = acc.n_over;
        pp.n_over[o] = 0;
        pp.n_lost[0] = acc.n_lost[0];
        pp.n_lost[1] = acc.n_lost[1];
    }
    // the last workgroup of the case finalises the step
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const unsigned prev = atomicAdd(&st->done, 1u);
        s_last = (prev + 1u == (unsigned)C->n_blocks);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    finish_ledger(C, st, P.partials, red);
    __syncthreads();
    const long long next = st->step + 1;
    solve_case(C, st, next + (kImp ? 1 : 0), DIAG, (double*)smem, red);
    if (tid == 0) {
        if (DIAG) st->eedf_samples += 1;
        st->step = next;
        st->done = 0u;
    }
}

template __global__ void k_step<0, false>(Params);
template __global__ void k_step<0, true>(Params);
template __global__ void k_step<1, false>(Params);
template __global__ void k_step<1, true>(Params);

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
    for (int i = start + (int)threadIdx.x; i < end; i += kBlock) {
        if (convert) {
            S.vx[i] = (float)((double)S.vx[i] * vs);
            S.vy[i] = (float)((double)S.vy[i] * vs);
            S.vz[i] = (float)((double)S.vz[i] * vs);
        }
        if (startup) {
            S.abar[i] = 0.0f;
            int c = S.cell[i];
            if (c < 0) continue;
            float o = S.off[i] + S.vx[i];
            renorm(c, o);
            if (C->bc == 1) {
                c %= N;
                if (c < 0) c += N;
            } else if (c < 0 || c >= N) {
                c = -1;
            }
            S.cell[i] = c;
            S.off[i] = o;
        }
    }
}

// ---------------------------------------------------------------------------
// Compaction: drop absorbed slots and sort every species by cell (a stable
// counting sort across workgroups; the order inside one cell is arbitrary).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_compact_hist(Params P, uint32_t* hist_all,
                                                         const int64_t* hist_off)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_lo, s_hi;
    const Work w = P.work[blockIdx.x];
    Case* C = P.cases + w.c;
    State* st = P.state + w.c;
    const Species& S = C->sp[w.s];
    const int N = C->n_cells;
    uint32_t* hist = hist_all + hist_off[2 * w.c + w.s];
    unsigned* lh = (unsigned*)smem;
    for (int j = threadIdx.x; j < N; j += kBlock) lh[j] = 0u;
    if (threadIdx.x == 0) {
        s_lo = kNoCell;
        s_hi = -1;
    }
    __syncthreads();
    const int n = st->n_slots[w.s];
    int chunk = (n + w.nb - 1) / w.nb;
    chunk = (chunk + 63) & ~63;
    const int start = w.b * chunk, end = min(n, start + chunk);
    int lo = kNoCell, hi = -1;
    for (int i = start + (int)threadIdx.x; i < end; i += kBlock) {
        const int c = S.cell[i];
        if (c >= 0) {
            atomicAdd(&lh[c], 1u);
            range_note(lo, hi, c);
        }
    }
    if (hi >= 0) {
        atomicMin(&s_lo, lo);
        atomicMax(&s_hi, hi);
    }
    __syncthreads();
    for (int j = s_lo + (int)threadIdx.x; s_hi >= 0 && j <= s_hi; j += kBlock)
        if (lh[j]) atomicAdd(&hist[j], lh[j]);
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
    const int N = C->n_cells;
    uint32_t* hist = hist_all + hist_off[2 * c + s];
    uint32_t* cur = cursor_all + hist_off[2 * c + s];
    unsigned* a = (unsigned*)smem;
    for (int j = threadIdx.x; j < N; j += kBlock) {
        a[j] = hist[j];
        hist[j] = 0u;
    }
    __syncthreads();
    block_scan(a, N, red);
    for (int j = threadIdx.x; j < N; j += kBlock) cur[j] = j > 0 ? a[j - 1] : 0u;
    if (threadIdx.x == 0) st->sort_live[s] = N > 0 ? a[N - 1] : 0;
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
    const Species& S = C->sp[w.s];
    const int N = C->n_cells;
    const bool imp = C->scheme == 1;
    uint32_t* cur = cursor_all + hist_off[2 * w.c + w.s];
    unsigned* lh = (unsigned*)smem;
    unsigned* lb = lh + N;
    for (int j = threadIdx.x; j < N; j += kBlock) lh[j] = 0u;
    if (threadIdx.x == 0) {
        s_lo = kNoCell;
        s_hi = -1;
    }
    __syncthreads();
    const int n = st->n_slots[w.s];
    int chunk = (n + w.nb - 1) / w.nb;
    chunk = (chunk + 63) & ~63;
    const int start = w.b * chunk, end = min(n, start + chunk);
    int lo = kNoCell, hi = -1;
    for (int i = start + (int)threadIdx.x; i < end; i += kBlock) {
        const int c = S.cell[i];
        if (c >= 0) {
            atomicAdd(&lh[c], 1u);
            range_note(lo, hi, c);
        }
    }
    if (hi >= 0) {
        atomicMin(&s_lo, lo);
        atomicMax(&s_hi, hi);
    }
    __syncthreads();
    for (int j = s_lo + (int)threadIdx.x; s_hi >= 0 && j <= s_hi; j += kBlock) {
        const unsigned k = lh[j];
        if (k) lb[j] = atomicAdd(&cur[j], k);
        lh[j] = 0u;
    }
    __syncthreads();
    double v2 = 0.0;
    for (int i = start + (int)threadIdx.x; i < end; i += kBlock) {
        const int c = S.cell[i];
        if (c < 0) continue;
        const unsigned d = lb[c] + atomicAdd(&lh[c], 1u);
        const float vx = S.vx[i], vy = S.vy[i], vz = S.vz[i];
        S.cell2[d] = c;
        S.off2[d] = S.off[i];
        S.vx2[d] = vx;
        S.vy2[d] = vy;
        S.vz2[d] = vz;
        S.id2[d] = S.id[i];
        float vh = vx;
        if (imp) {
            const float ab = S.abar[i];
            S.abar2[d] = ab;
            vh = vx - 0.5f * ab;   // v_{n-1/2} from the stored prediction
        }
        v2 += (double)(vh * vh + vy * vy + vz * vz);
    }
    v2 = block_sum(v2, red);
    if (threadIdx.x == 0) P.partials[blockIdx.x].v2sum[w.s] = v2;
}

// one workgroup per case: swap buffers, set counts and the exact kinetic energy
__global__ __launch_bounds__(kBlock) void k_compact_finish(Params P)
{
    __shared__ double red[kWaves];
    Case* C = P.cases + blockIdx.x;
    State* st = P.state + blockIdx.x;
    const int nb = C->n_blocks, fb = C->first_block;
    for (int s = 0; s < 2; ++s) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nb; b += kBlock) {
            const Work w = P.work[fb + b];
            if (w.s == s) v += P.partials[fb + b].v2sum[s];
        }
        v = block_sum(v, red);
        if (threadIdx.x == 0) {
            Species& S = C->sp[s];
            st->K[s] = v * S.kin_unit;
            st->sortK[s] = st->K[s];
            const int live = (int)st->sort_live[s];
            st->n_slots[s] = live;
            st->n_live[s] = live;
            int32_t* t0 = S.cell; S.cell = S.cell2; S.cell2 = t0;
            float* t1 = S.off; S.off = S.off2; S.off2 = t1;
            t1 = S.vx; S.vx = S.vx2; S.vx2 = t1;
            t1 = S.vy; S.vy = S.vy2; S.vy2 = t1;
            t1 = S.vz; S.vz = S.vz2; S.vz2 = t1;
            uint64_t* t2 = S.id; S.id = S.id2; S.id2 = t2;
            t1 = S.abar; S.abar = S.abar2; S.abar2 = t1;
        }
        __syncthreads();
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
    for (int j = threadIdx.x; j < N; j += kBlock) dep[j] = 0ull;
    if (threadIdx.x == 0) {
        s_lo = kNoCell;
        s_hi = -1;
    }
    __syncthreads();
    const int n = st->n_slots[w.s];
    int chunk = (n + w.nb - 1) / w.nb;
    chunk = (chunk + 63) & ~63;
    const int start = w.b * chunk, end = min(n, start + chunk);
    int lo = kNoCell, hi = -1;
    for (int i = start + (int)threadIdx.x; i < end; i += kBlock) {
        const int c = S.cell[i];
        if (c < 0) continue;
        atomicAdd(&dep[c], packw(S.off[i]));
        range_note(lo, hi, c);
    }
    if (hi >= 0) {
        atomicMin(&s_lo, lo);
        atomicMax(&s_hi, hi);
    }
    __syncthreads();
    for (int j = s_lo + (int)threadIdx.x; s_hi >= 0 && j <= s_hi; j += kBlock) {
        const unsigned long long p = dep[j];
        if (p) {
            atomicAdd(&C->dep_cnt[w.s][j], p >> 40);
            atomicAdd(&C->dep_w[w.s][j], p & kWMask);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_solve(Params P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kWaves];
    Case* C = P.cases + blockIdx.x;
    State* st = P.state + blockIdx.x;
    solve_case(C, st, st->step + (C->scheme == 1 ? 1 : 0), false, (double*)smem, red);
}

}  // namespace pic
