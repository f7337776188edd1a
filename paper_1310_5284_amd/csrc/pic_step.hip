// HIP kernels of the particle step of the EC PIC/MCC method for gfx950
// (MI355X): k_step, the streaming pass over the particle arrays of every
// case of a scheme (gather, push, boundary, waiting-time candidacy,
// privatised deposit, candidate list), and k_collide, the null-collision MCC
// of the listed candidates (with the implicit prediction and ionization
// children).  The method:
//   - charge weighting, Sec. II Eq. (2): S_1 (m = 1) or S_2 (m = 2)
//   - field interpolation, Sec. II Eq. (3): S_0 (m = 1) or S_1 (m = 2) of the
//     half-grid field (EC), or linear of the nodal field (MC, scheme (1))
//   - explicit leap-frog / D1 direct-implicit push, Sec. II schemes (1)-(4)
//   - absorbing electrodes, RF bias, MCC with the gas, Sec. III
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "pic.h"
#include "pic_common.hpp"
#include "pic_device.hpp"
#include "pic_weights.hpp"

namespace pic {

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
// children, and the undoing of a null prediction after a real collision of
// an implicit particle; both rare): linear (count and weight of its cell) or
// quadratic, with the susceptibility word of the m = 2 implicit scheme.
// remove: take the particle's words out again (the same integers).
__device__ __forceinline__ void deposit_global(const Case* C, int s, int c, float o,
                                               bool remove = false)
{
    PIC_GLOBAL unsigned long long* gcnt = gp(C->dep_cnt[s]);
    PIC_GLOBAL unsigned long long* gw = gp(C->dep_w[s]);
    auto add = [&](PIC_GLOBAL unsigned long long* a, unsigned long long v) {
        gatomic_add(a, remove ? 0ull - v : v);
    };
    const int N = C->n_cells;
    const bool periodic = C->bc == 1;
    if (C->gather == 2 && C->scheme == 1) {
        // the moment form of deposit_moments: counts and sums of node i
        uint32_t w[3];
        int i = quad_weights(c, o, w);
        if (periodic && i == N) i = 0;
        const bool left = o >= 0.5f;
        add(&gcnt[i], left ? 0ull : 1ull);
        add(&gw[i], (unsigned long long)w[0]);
        add(gp(&C->chi_cnt[s][i]), left ? 1ull : 0ull);
        add(gp(&C->chi_w[s][i]), (unsigned long long)w[2]);
        if (C->chl_w0[s] && left) {   // nonuniform grid: the left-side sums
            add(gp(&C->chl_w0[s][i]), (unsigned long long)w[0]);
            add(gp(&C->chl_w2[s][i]), (unsigned long long)w[2]);
        }
        return;
    }
    if (C->gather == 2) {
        uint32_t w[3];
        const int i = quad_weights(c, o, w);
        for (int k = 0; k < 3; ++k)
            add(&gw[fold_node(i - 1 + k, N, periodic)], (unsigned long long)w[k]);
    } else {
        add(&gw[c], packw(o) & kWMask);
    }
    add(&gcnt[c], 1ull);
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
//   x~' = x + v~', absorb and deposit x~'.  Subcycled ions move only in the
//   steps n % K == 0, with K dt: x = x~ + K^2 a/2, v = v~ + K a/2,
//   v~' = v + K abar/2, x~' = x + K v~'.
//
// The streaming loop issues the loads of kILP particles per thread together
// (indices past the chunk are clamped to its last slot and treated as dead).
// Candidates store x_{n+1} and are listed (slot, v_{n+1/2}, abar_n) in the
// region of the workgroup's chunk for k_collide (ballot + one LDS atomic per
// wavefront).  The deposit goes to a privatised LDS grid (one int64 per cell
// packs count and summed weight), flushed over the cell range the workgroup
// touched.  The workgroup's ledger partial is a row of plain stores.
// ---------------------------------------------------------------------------
// Launch variants by what the cases of a batch need, so that no kernel
// carries code its cases cannot reach (a shorter kernel measured faster):
// PLAIN: every case has the EC gather (m = 1) on a uniform grid.  DUAL: the
// moment words of m = 2 implicit are compiled in.  GT: the width ratios and
// runs of nonuniform grids are read from global memory (cached) instead of
// LDS: the variant for batches with an m = 2 implicit case on a nonuniform
// grid, whose four moment words per node would otherwise leave one
// workgroup per CU.
template <int SCHEME, bool DIAG, bool GT, bool DUAL, bool PLAIN>
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
    const bool mc = !PLAIN && C->gather == 1;
    // (an implicit m = 2 case is launched only in the DUAL variant)
    const bool ec2 = !PLAIN && C->gather == 2 && (!kImp || DUAL);
    const bool dual = DUAL && kImp && ec2;   // susceptibility words of its own
    const bool nu = !PLAIN && C->nonuniform != 0;
    const bool coll = C->collisions != 0 && C->sp[s].n_proc > 0;

    const StepLds L = step_lds_layout(N, DIAG, dual, nu, !GT);
    float* eh = (float*)smem;
    unsigned long long* dep = (unsigned long long*)(smem + L.dep);
    unsigned long long* dch = (unsigned long long*)(smem + L.dual);
    // m = 2 implicit on a nonuniform grid: the left-side P0 and P2 sums
    const bool duo = dual && nu;
    unsigned long long* dl0 =
        duo ? (unsigned long long*)(smem + L.dual + align16(8 * ((size_t)N + 1))) : nullptr;
    unsigned long long* dl2 =
        duo ? (unsigned long long*)(smem + L.dual + 2 * align16(8 * ((size_t)N + 1))) : nullptr;
    // nonuniform: dx / w_c and the runs of equal widths
    using RT = typename std::conditional<GT, const PIC_GLOBAL float*, float*>::type;
    using UT = typename std::conditional<GT, const PIC_GLOBAL uint32_t*, uint32_t*>::type;
    RT rl;
    UT ul;
    if constexpr (GT) {
        rl = gp((const float*)C->cell_r);
        ul = gp((const uint32_t*)C->cell_run);
    } else {
        rl = (float*)(smem + L.ratio);
        ul = (uint32_t*)(smem + L.ratio + align16(4 * (size_t)N));
    }
    float* heat = (float*)(smem + L.heat);
    unsigned* eedf = (unsigned*)(smem + L.eedf);
    {
        const PIC_GLOBAL float* ehg = gp(C->ehat[s]);
        if (mc) {
            if (nu) {
                const PIC_GLOBAL float* rg = gp(C->cell_r);
                for (int g = tid; g <= N; g += kBlock) eh[g] = nodal_field_nu(ehg, rg, N, g);
            } else {
                for (int g = tid; g <= N; g += kBlock) eh[g] = nodal_field(ehg, N, periodic, g);
            }
        } else if (ec2 && nu) {
            // m = 2 on a nonuniform grid: the potential differences E w_j
            // (in units of dx) are interpolated, and the result divided by
            // the width of the particle's cell (minus the physical gradient
            // of the deposit's field energy)
            const PIC_GLOBAL float* rg = gp(C->cell_r);
            for (int j = tid; j < N; j += kBlock) eh[j] = ehg[j] / rg[j];
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
    if (dual)
        for (int j = tid; j <= N; j += kBlock) {
            dch[j] = 0ull;
            if (duo) {
                dl0[j] = 0ull;
                dl2[j] = 0ull;
            }
        }
    if constexpr (!GT) {
        if (nu) {
            const PIC_GLOBAL float* rg = gp(C->cell_r);
            const PIC_GLOBAL uint32_t* ug = gp(C->cell_run);
            for (int j = tid; j < N; j += kBlock) {
                rl[j] = rg[j];
                ul[j] = ug[j];
            }
        }
    }
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
    // subcycled ions stand in the steps between their pushes (the workgroup
    // still writes its zero ledger row and empty list); a push takes K dt
    const int ksub = s == 1 ? C->ion_sub : 1;
    const bool stands = ksub > 1 && (st->step % ksub) != 0;
    const float kf = (float)ksub;
    const float hk = 0.5f * kf, hk2 = hk * kf;   // D1 with the step K dt: K/2, K^2/2
    const uint32_t clk = clock_from(st->step, ksub, coll);   // the species' clock
    const int end = stands ? start : min(n, start + chunk);

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
                             : (ec2 ? gather_ec2(eh, N, periodic, cc, o[k]) * (nu ? rl[cc] : 1.0f)
                                    : eh[cc]);
            float vn, vold, abn = 0.0f, o1, mv;
            if (kImp) {
                vold = v[k] - hk * ab[k];
                vn = v[k] + hk * a;
                abn = 0.5f * (ab[k] + a);
                mv = hk2 * a;
            } else {
                vold = v[k];
                vn = fmaf(kf, a, v[k]);   // kf = 1 but for subcycled ions
                mv = kf * vn;
            }
            o1 = o[k] + mv;
            int c1 = cc;
            if (live) {
                const float dk = (vn - vold) * (vn + vold);
                wk += dk;
                if (DIAG) {
                    atomicAdd(&heat[cc], dk);
                    range_note(lo, hi, cc);
                }
                if (nu) {
                    o1 = o[k];
                    walk(c1, o1, mv, rl, ul, N);
                } else {
                    renorm(c1, o1);
                }
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
            const bool isc = live && coll && wait_count(wt, clk) == 0u;
            // non-candidates finish here; candidates store x_{n+1} (final
            // for the explicit scheme, which deposits it now) but not their
            // cell word, which k_collide writes with the next waiting time
            int c2 = c1;
            float o2 = o1, vst = vn;
            bool dep_now = false;
            uint32_t lflag = 0u;   // list flag of a candidate
            if (live && !isc) {
                if (kImp) {
                    vst = nu ? predict_nu(c2, o2, vn, abn, rl, ul, N, kf)
                             : predict(c2, o2, vn, abn, kf);
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
                    // the word changes only with the cell (the waiting-time
                    // field is an expiry)
                    if (c2 != cc) stg(cellp, i4, pack_cell(c2, wt));
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
                    const float vp = nu ? predict_nu(cp, op, vn, abn, rl, ul, N, kf)
                                        : predict(cp, op, vn, abn, kf);
                    if (periodic) {
                        cp %= N;
                        if (cp < 0) cp += N;
                    }
                    if (cp >= 0 && cp < N) {
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
                    stg(offp, i4, o1);
                    // explicit: v_{n+1/2} stands unless k_collide finds a
                    // real collision (the store joins the coalesced stream)
                    if (!kImp) stg(vxp, i4, vn);
                }
                dep_now = !kImp || kept;
            }
            if (dual)
                deposit_moments(dep, dch, dep_now, c2, o2, N, periodic, lo, hi, s == 1, dl0, dl2);
            else if (ec2)
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
                    // the list word carries the capped flag and the
                    // prediction flag in its waiting-time field
                    stg(cq_w, e4, pack_cell(c1, (wt & PIC_WAIT_CAPPED) | lflag));
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
            if (dual) {
                const unsigned long long d = dch[j];
                if (d) {
                    gatomic_add(gp(&C->chi_cnt[s][j]), d >> 40);
                    gatomic_add(gp(&C->chi_w[s][j]), d & kWMask);
                }
                if (duo) {
                    if (dl0[j]) gatomic_add(gp(&C->chl_w0[s][j]), dl0[j]);
                    if (dl2[j]) gatomic_add(gp(&C->chl_w2[s][j]), dl2[j]);
                }
            }
            // the range covers nodes (up to N for the quadratic deposit);
            // the heating profile has the N cells only
            if (DIAG && j < N) {
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
// (at most 128 VGPRs: 4 wavefronts per SIMD; it fits without spilling)
// DUAL, PLAIN: the launch variants of k_step.
template <int SCHEME, bool DIAG, bool DUAL, bool PLAIN>
__global__ __launch_bounds__(kBlock, 4) void k_collide(Params P)
{
    const CollideWork cw = P.cwork[P.mode + (int)blockIdx.x];
    const int gblk = cw.step_blk;
    // the list's length is checked after the case's loads have been issued
    // beside its load
    const int ncand = P.cand_n[gblk];
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ BlockAcc acc;
    __shared__ Species S;
    __shared__ ChildEv cq[kChildQ];
    __shared__ int q_n;
    constexpr bool kImp = SCHEME == 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const Work w = cw.w;
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
    // (an implicit m = 2 case is launched only in the DUAL variant)
    const bool ec2 = !PLAIN && C->gather == 2 && (!kImp || DUAL);
    const bool dual = kImp && ec2;   // susceptibility words of its own
    const bool nu = !PLAIN && C->nonuniform != 0;
    const PIC_GLOBAL float* rg = gp(uniform_ptr((const float*)C->cell_r));   // nu: dx / w_c
    const PIC_GLOBAL uint32_t* ug = gp(uniform_ptr((const uint32_t*)C->cell_run));   // and runs
    const uint32_t k0 = C->key0, k1 = C->key1;
    const CollideLds L = collide_lds_layout(N, dual, nu);
    unsigned long long* dep = (unsigned long long*)smem;
    unsigned long long* dch = (unsigned long long*)(smem + L.dual);
    const bool duo = dual && nu;   // the left-side sums (nonuniform grid)
    unsigned long long* dl0 =
        duo ? (unsigned long long*)(smem + L.dual + align16(8 * ((size_t)N + 1))) : nullptr;
    unsigned long long* dl2 =
        duo ? (unsigned long long*)(smem + L.dual + 2 * align16(8 * ((size_t)N + 1))) : nullptr;
    unsigned* eedf = (unsigned*)(smem + L.eedf);
    __shared__ float lbound[kBoundBins];
    if (s == 0 && C->sp[0].n_proc > 0)
        for (int j = tid; j < kBoundBins; j += kBlock) lbound[j] = C->sp[0].cbound[j];
    if (kImp)
        for (int j = tid; j <= N; j += kBlock) {
            dep[j] = 0ull;
            if (dual) dch[j] = 0ull;
            if (duo) {
                dl0[j] = 0ull;
                dl2[j] = 0ull;
            }
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
        q_n = 0;
    }
    if (cw.round * kBlock >= ncand) return;   // nothing in this round
    lds_barrier();

    const uint32_t step32 = (uint32_t)st->step;
    // the species' clock after this step, and the children's clocks
    const int ksub = s == 1 ? C->ion_sub : 1;
    // (k_collide runs only for species with trials; an ion species without a
    // process keeps its clock at 0)
    const uint32_t clk1 = clock_from(st->step, ksub, true) + 1u;
    const float kf = (float)ksub;   // the species' D1 step in units of dt
    // implicit: an ion child is predicted with the ions' step when the ions
    // move in this step; otherwise it stands where it was created
    const bool ions_move = C->ion_sub <= 1 || st->step % C->ion_sub == 0;
    const float kfi = ions_move ? (float)C->ion_sub : 0.0f;
    const uint32_t clk_e = clock_from(st->step + 1, 1, true),
                   clk_i = clock_from(st->step + 1, C->ion_sub, C->sp[1].n_proc > 0);
    const int ns0 = st->n_slots[0], ns1 = st->n_slots[1];
    const int n = st->n_slots[s];
    int chunk = (n + w.nb - 1) / w.nb;
    chunk = (chunk + 63) & ~63;
    const int region = w.b * chunk;   // the candidate list of this workgroup
    const float eedf_k = S.eps_unit * S.eedf_scale;
    // stores of a candidate's new state, with the context's store policy:
    // the default one leaves the lines in the caches for the next step's
    // pass, the non-temporal one keeps them from evicting what that pass
    // reads; which is faster depends on the workload (the autotuner measures)
    const bool nts = P.nt_store != 0;
    auto put = [&](auto* base, uint32_t off, auto v) {
        if (nts) stg_nt(base, off, v);
        else stg(base, off, v);
    };

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
                if (nu) {
                    walk(ce, oe, ch.vx, rg, ug, N);
                    if (kfi > 0.0f) walk(ci, oi, kfi * ch.ix, rg, ug, N);
                } else {
                    oe = o1 + ch.vx;
                    renorm(ce, oe);
                    oi = o1 + kfi * ch.ix;
                    renorm(ci, oi);
                }
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
                               wait_field(clk_e, wait_encode(geo0(r4.x, S.inv_log1mp))), kImp);
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
                               wait_field(clk_i, wait_encode(geo0(r4.x, inv_ion))), kImp);
                deposit_global(C, 1, ci, oi);
            } else {
                atomicAdd(&acc.n_lost[1], 1u);
            }
        }
    };

    // the rounds of a list take its blocks of kBlock candidates in turn, so
    // a thread's candidates follow at a stride of rounds * kBlock.  A dense
    // list gives a thread many of them: the next one's list entries and
    // record, and the slot of the one after, are loaded while the current
    // one is processed (one candidate ahead: more ahead measured slower on
    // sparse lists, where a thread has one candidate and the registers cost
    // occupancy)
    struct Pay {
        u32x4 r;   // the 16-byte record: id, vy, vz
        float vn, ab, o;
        int32_t w;
    };
    auto load_pay = [&](int e, int i) {
        Pay p;
        const uint32_t q4 = (uint32_t)(region + e) << 2;
        p.vn = ldg(cq_vn, q4);
        p.ab = kImp ? ldg(cq_ab, q4) : 0.0f;
        // the list carries x_{n+1}
        p.w = ldg(cq_w, q4);
        p.o = kImp ? ldg(cq_o, q4) : 0.0f;
        // a candidate's record is one scattered 16-byte read: loaded with
        // the non-temporal policy, which on gfx950 moves about half the
        // bytes of a cached line fill for such reads
        p.r = ldg_nt((const PIC_GLOBAL u32x4*)recp, (uint32_t)i << 4);
        return p;
    };
    const int estep = cw.rounds * kBlock;
    int i_nx = 0, i_nx2 = 0;
    Pay p_nx{};
    {
        const int ef = cw.round * kBlock + tid;
        if (ef < ncand) {
            i_nx = ldg(cq_idx, (uint32_t)(region + ef) << 2);
            p_nx = load_pay(ef, i_nx);
        }
        if (ef + estep < ncand) i_nx2 = ldg(cq_idx, (uint32_t)(region + ef + estep) << 2);
    }
    for (int e0 = cw.round * kBlock; e0 < ncand; e0 += estep) {
        const int e = e0 + tid;
        const bool act = e < ncand;
        const Pay pc = p_nx;
        int i = i_nx, c1 = 0;
        if (e + estep < ncand) {
            i_nx = i_nx2;
            p_nx = load_pay(e + estep, i_nx);
        }
        if (e + 2 * estep < ncand) i_nx2 = ldg(cq_idx, (uint32_t)(region + e + 2 * estep) << 2);
        float o1 = 0.0f, vn = 0.0f, vn0 = 0.0f, abn = 0.0f, vy = 0.0f, vz = 0.0f;
        uint64_t id = 0;
        bool pred = false;  // implicit: k_step deposited the null prediction
        uint32_t nw = 0u;   // the particle's next waiting-time word
        int kind = -1;
        Child ch;
        if (act) {
            vn = pc.vn;
            if (kImp) abn = pc.ab;
            const uint32_t i4 = (uint32_t)i << 2;
            const int32_t w1 = pc.w;
            if (kImp) o1 = pc.o;
            const u32x4 r = pc.r;
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
                    nw = wait_field(clk1, wait_encode(W - 1.0));
                }
            }
            if (is_cand) {
                const uint4 r0 = philox((uint32_t)id, (uint32_t)(id >> 32), step32,
                                        (uint32_t)s << 28, k0, k1);
                ++cand;
                nw = wait_field(clk1, wait_encode(geo0(r0.x, S.inv_log1mp)));
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
                put((PIC_GLOBAL u32x2*)recp, (i4 << 2) + 8u, yz);
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
                if (nu) predict_nu(c2, o2, vn, abn, rg, ug, N, kf);
                else predict(c2, o2, vn, abn, kf);
                if (periodic) {
                    c2 %= N;
                    if (c2 < 0) c2 += N;
                }
                put(cellp, i4, pack_cell(c2, nw));
            } else if (kImp) {
                if (pred) {
                    // a real collision: undo k_step's deposit of the null
                    // prediction (integer words, so exactly)
                    int cp = c1;
                    float op = o1;
                    if (nu) predict_nu(cp, op, vn0, abn, rg, ug, N, kf);
                    else predict(cp, op, vn0, abn, kf);
                    if (periodic) {
                        cp %= N;
                        if (cp < 0) cp += N;
                    }
                    if (ec2) {
                        deposit_global(C, s, cp, op, true);
                    } else {
                        gatomic_add(&gdep_cnt[cp], ~0ull);
                        gatomic_add(&gdep_w[cp], 0ull - (packw(op) & kWMask));
                    }
                }
                const float vst = nu ? predict_nu(c2, o2, vn, abn, rg, ug, N, kf)
                                     : predict(c2, o2, vn, abn, kf);
                bool gone = false;
                if (periodic) {
                    c2 %= N;
                    if (c2 < 0) c2 += N;
                } else if (c2 < 0 || c2 >= N) {
                    absorb(i, c2 < 0 ? 0 : 1, vn, vy, vz);
                    gone = true;
                }
                if (!gone) {
                    put(cellp, i4, pack_cell(c2, nw));
                    put(offp, i4, o2);
                    put(vxp, i4, vst);
                    put(abp, i4, abn);
                    dep_ok = true;
                }
            } else {
                if (kind >= 0) put(vxp, i4, vn);   // the pass stored v_{n+1/2}
                put(cellp, i4, pack_cell(c1, nw));
            }
        }
        if (kImp) {
            if (ec2) {
                deposit_moments(dep, dch, dep_ok, c2, o2, N, periodic, lo, hi, false, dl0, dl2);
            } else {
                deposit_wave(dep, dep_ok, c2, o2, lo, hi);
            }
        }
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
            if (dual) {
                const unsigned long long d = dch[j];
                if (d) {
                    gatomic_add(gp(&C->chi_cnt[s][j]), d >> 40);
                    gatomic_add(gp(&C->chi_w[s][j]), d & kWMask);
                }
                if (duo) {
                    if (dl0[j]) gatomic_add(gp(&C->chl_w0[s][j]), dl0[j]);
                    if (dl2[j]) gatomic_add(gp(&C->chl_w2[s][j]), dl2[j]);
                }
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

template __global__ void k_step<0, false, false, false, true>(Params);
template __global__ void k_step<0, true, false, false, true>(Params);
template __global__ void k_step<0, false, false, false, false>(Params);
template __global__ void k_step<0, true, false, false, false>(Params);
template __global__ void k_step<1, false, false, false, true>(Params);
template __global__ void k_step<1, true, false, false, true>(Params);
template __global__ void k_step<1, false, false, false, false>(Params);
template __global__ void k_step<1, true, false, false, false>(Params);
template __global__ void k_step<1, false, false, true, false>(Params);
template __global__ void k_step<1, true, false, true, false>(Params);
template __global__ void k_step<1, false, true, true, false>(Params);
template __global__ void k_step<1, true, true, true, false>(Params);
template __global__ void k_collide<0, false, false, false>(Params);
template __global__ void k_collide<0, true, false, false>(Params);
template __global__ void k_collide<1, false, false, true>(Params);
template __global__ void k_collide<1, true, false, true>(Params);
template __global__ void k_collide<1, false, false, false>(Params);
template __global__ void k_collide<1, true, false, false>(Params);
template __global__ void k_collide<1, false, true, false>(Params);
template __global__ void k_collide<1, true, true, false>(Params);

}  // namespace pic
