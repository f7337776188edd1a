// Plain FP64 GPU form of the EC PIC/MCC step: the comparison point of the
// throughput metric.  The same method as k_step / k_collide (Sec. II,
// Eqs. (2)-(3), schemes (1)-(4); Sec. III), written the straightforward way:
// float64 absolute positions xi = x/dx and velocities, one launch per phase
// (deposit, solve, push+MCC), float64 global atomics for the deposit (and the
// cell counts of the implicit susceptibility), no sorting, no privatisation,
// children appended with one atomic each, absorbed particles flagged dead.
// Explicit leap-frog and the D1 direct-implicit scheme (beta = 1/2), EC and
// MC gathers, with an energy ledger per step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "pic.h"
#include "pic_common.hpp"
#include "pic_device.hpp"

namespace pic {

struct Species64 {
    double* xi;
    double* vx;
    double* vy;
    double* vz;
    double* abar;       // D1: the averaged acceleration (cells/step^2)
    uint64_t* id;
    int32_t* alive;
    uint32_t* wait;     // null-collision waiting-time words
    int64_t capacity;
    double accel;       // cells/step^2 per (V/m)
    double qw_dx;
    double kin_unit;    // J/m^2 per unit v^2
    double chi_coef;    // beta dt^2 q^2 w / (m eps0 dx) per particle in a cell
    double eps_unit, t_scale, t_off, t_max;
    double thr_v2[kMaxProc];
    int32_t kind[kMaxProc];
    int32_t n_proc;
    uint32_t cand_thr;
    double inv_log1mp;  // 1 / ln(1 - P_null)
    double vth_neutral, vth_newion, recoil2, opal_B;
    const double* tab;  // electrons [n][4], ions [n]: sigma * n_g (dx/dt) / nu_max
};

struct Case64 {
    int32_t n_cells, bc, gather, collisions, scheme, pad;
    double dx, dt, rf_volts, rf_omega, background_rho;
    uint32_t key0, key1;
    Species64 sp[2];
    double* Q[2];     // [N+1] linear node weights
    double* cnt[2];   // [N] particles per cell (implicit EC susceptibility)
    double* E;        // [N]
    double* phi;      // [N+1]
};

// Ledger of one step (J/m^2 and counts), accumulated by the push kernel.
struct Led64 {
    double K_before[2], K_after[2], work[2], coll[2], absK[2][2], WE;
    unsigned long long abs_n[2][2], n_coll[2][4], n_cand[2], n_created[2], n_over[2];
};

struct State64 {
    long long step;       // index of the next solve
    long long step_push;  // index of the running push
    int32_t n_cur[2];     // slots pushed this step
    int32_t n_next[2];    // slots after appends
    int32_t lost[2];
    Led64 led;            // the running step's ledger (the last step's after a call)
};

struct Params64 {
    Case64* cases;
    State64* state;
    const Work* work;
};

__device__ __forceinline__ double u01d(uint32_t r)
{
    return (double)((r >> 9) * 2u + 1u) * 5.9604644775390625e-08;
}

__global__ __launch_bounds__(kBlock) void k64_deposit(Params64 P)
{
    const Work w = P.work[blockIdx.x];
    Case64* C = P.cases + w.c;
    const Species64& S = C->sp[w.s];
    const bool counts = C->scheme == 1 && C->gather == 0;
    const int n = P.state[w.c].n_next[w.s];
    int chunk = (n + w.nb - 1) / w.nb;
    chunk = (chunk + 63) & ~63;
    const int start = w.b * chunk, end = min(n, start + chunk);
    for (int i = start + (int)threadIdx.x; i < end; i += kBlock) {
        if (!S.alive[i]) continue;
        const double x = S.xi[i];
        const double j = floor(x);
        const double f = x - j;
        const int jj = (int)j;
        atomicAdd(&C->Q[w.s][jj], 1.0 - f);
        atomicAdd(&C->Q[w.s][jj + 1], f);
        if (counts) atomicAdd(&C->cnt[w.s][jj], 1.0);
    }
}

// One workgroup per case: rho from the deposits, the susceptibility of the
// implicit scheme, the first-integral solve, E; opens the step's ledger.
__global__ __launch_bounds__(kBlock) void k64_solve(Params64 P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kWaves];
    Case64* C = P.cases + blockIdx.x;
    State64* st = P.state + blockIdx.x;
    const int N = C->n_cells, tid = threadIdx.x;
    const bool periodic = C->bc == 1;
    const bool implicit = C->scheme == 1;
    const double dx = C->dx;
    const double eps0 = 8.8541878128e-12;
    double* S = (double*)smem;         // [N+1] node charges, then R_j
    double* K = S + (N + 1);           // [N] eps0 (1 + chi_j)
    for (int g = tid; g <= N; g += kBlock) {
        double r = C->background_rho;
        for (int s = 0; s < 2; ++s) {
            double q = C->Q[s][g];
            if (periodic && (g == 0 || g == N)) q = C->Q[s][0] + C->Q[s][N];
            r += C->sp[s].qw_dx * q;
        }
        S[g] = r;
    }
    for (int j = tid; j < N; j += kBlock) {
        double chi = 0.0;
        if (implicit) {
            for (int s = 0; s < 2; ++s) {
                if (C->gather == 0) {
                    chi += C->sp[s].chi_coef * C->cnt[s][j];
                } else {
                    // mean of the two node susceptibilities of the linear
                    // weights over the node volumes (half a cell at an electrode)
                    double ql = C->Q[s][j], qr = C->Q[s][j + 1];
                    if (periodic) {
                        if (j == 0) ql = C->Q[s][0] + C->Q[s][N];
                        if (j + 1 == N) qr = C->Q[s][0] + C->Q[s][N];
                    }
                    const double vl = (!periodic && j == 0) ? 0.5 : 1.0;
                    const double vr = (!periodic && j + 1 == N) ? 0.5 : 1.0;
                    chi += 0.5 * C->sp[s].chi_coef * (ql / vl + qr / vr);
                }
            }
        }
        K[j] = eps0 * (1.0 + chi);
    }
    __syncthreads();
    for (int g = tid; g <= N; g += kBlock) {
        C->Q[0][g] = 0.0;
        C->Q[1][g] = 0.0;
        if (g < N && implicit && C->gather == 0) {
            C->cnt[0][g] = 0.0;
            C->cnt[1][g] = 0.0;
        }
    }
    if (tid == 0) S[0] = 0.0;
    __syncthreads();
    for (int k = 1 + tid; k < N; k += kBlock) S[k] *= dx;
    __syncthreads();
    block_scan(S, N, red);
    // D_{j+1/2} = D0 + R_j, E = D / (eps0 (1 + chi)), sum_j E dx = V
    double a = 0.0, b = 0.0;
    for (int j = tid; j < N; j += kBlock) {
        a += S[j] / K[j];
        b += 1.0 / K[j];
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    const long long step = st->step;
    const long long field_step = implicit ? step + 1 : step;
    const double V =
        periodic ? 0.0 : C->rf_volts * sin(C->rf_omega * ((double)field_step * C->dt));
    const double D0 = (V / dx - a) / b;
    double we = 0.0;
    for (int j = tid; j < N; j += kBlock) {
        const double E = (D0 + S[j]) / K[j];
        C->E[j] = E;
        we += 0.5 * eps0 * E * E * dx;
    }
    we = block_sum(we, red);
    if (tid == 0) {
        st->step_push = step;
        st->step = step + 1;
        st->n_cur[0] = st->n_next[0];
        st->n_cur[1] = st->n_next[1];
        // the ledger of the step about to be pushed
        Led64& L = st->led;
        const double k0 = L.K_after[0], k1 = L.K_after[1];
        memset(&L, 0, sizeof(Led64));
        L.K_before[0] = k0;
        L.K_before[1] = k1;
        L.WE = we;
    }
}

// Boundary rule: absorbed outside [0, N) (Dirichlet), wrapped (periodic).  A
// non-finite position is removed so that no index is ever formed from it.
__device__ __forceinline__ void renorm64(double& x, int N, bool periodic, bool& absorbed)
{
    absorbed = false;
    if (!isfinite(x)) {
        absorbed = true;
        return;
    }
    if (periodic) {
        x -= (double)N * floor(x / (double)N);
        if (x >= (double)N) x -= (double)N;
        if (x < 0.0) x = 0.0;
    } else if (x < 0.0 || x >= N) {
        absorbed = true;
    }
}

__device__ __forceinline__ void iso_dir64(double ua, double ub, double& dx, double& dy, double& dz)
{
    const double ct = 1.0 - 2.0 * ua;
    const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double sp, cp;
    sincospi(2.0 * ub, &sp, &cp);
    dx = st * cp;
    dy = st * sp;
    dz = ct;
}

__device__ __forceinline__ void box_muller64(double ua, double ub, double& n1, double& n2)
{
    const double r = sqrt(-2.0 * log(ua));
    double sp, cp;
    sincospi(2.0 * ub, &sp, &cp);
    n1 = r * cp;
    n2 = r * sp;
}

__device__ __forceinline__ uint32_t geo_wait64(uint32_t r, double inv)
{
    const double W = floor(log(u01d(r)) * inv);
    return W > (double)PIC_WAIT_MAX ? (PIC_WAIT_MAX | PIC_WAIT_CAPPED) : (uint32_t)W;
}

// Per-thread ledger terms of a push workgroup (species s): the workgroup sums
// them and adds them to the case's ledger with one atomic each.
enum { A_WORK, A_KAFT, A_COLL, A_ABS0, A_ABS1, A_COLL_O, A_KAFT_O, A_ABS0_O, A_ABS1_O, A_ND };
enum { C_ABS0, C_ABS1, C_COLL0, C_COLL1, C_COLL2, C_COLL3, C_CAND, C_CRE0, C_CRE1, C_ABS0_O,
       C_ABS1_O, C_OVER, C_NU };

// A child at x (cells) appended to species cs; implicit children are
// predicted with abar = 0 (x~ = x + v) and absorbed there if outside.
__device__ __forceinline__ void append64(Case64* C, State64* st, int cs, int ps, double x,
                                         double vx, double vy, double vz, uint64_t id,
                                         uint32_t step, uint32_t k0, uint32_t k1, double* ad,
                                         unsigned* ac)
{
    const Species64& S = C->sp[cs];
    const bool own = cs == ps;
    const double ke = S.kin_unit * (vx * vx + vy * vy + vz * vz);
    ad[own ? A_COLL : A_COLL_O] += ke;
    ad[own ? A_KAFT : A_KAFT_O] += ke;
    ac[cs == 0 ? C_CRE0 : C_CRE1] += 1u;
    if (C->scheme == 1) {
        x += vx;
        bool gone;
        renorm64(x, C->n_cells, C->bc == 1, gone);
        if (gone) {
            const int e = x < 0.0 ? 0 : 1;
            ad[own ? A_KAFT : A_KAFT_O] -= ke;
            ad[(own ? A_ABS0 : A_ABS0_O) + e] += ke;
            ac[(own ? C_ABS0 : C_ABS0_O) + e] += 1u;
            return;
        }
    }
    const int slot = atomicAdd(&st->n_next[cs], 1);
    if (slot >= S.capacity) {
        atomicAdd(&st->lost[cs], 1);
        atomicSub(&st->n_next[cs], 1);
        return;
    }
    S.xi[slot] = x;
    S.vx[slot] = vx;
    S.vy[slot] = vy;
    S.vz[slot] = vz;
    S.abar[slot] = 0.0;
    S.id[slot] = id;
    S.alive[slot] = 1;
    // first trial of the child at the next step: draw 4 of its stream
    const uint4 r4 = philox((uint32_t)id, (uint32_t)(id >> 32), step, ((uint32_t)cs << 28) | 4u,
                            k0, k1);
    S.wait[slot] = geo_wait64(r4.x, S.inv_log1mp);
}

__global__ __launch_bounds__(kBlock) void k64_push(Params64 P)
{
    const Work w = P.work[blockIdx.x];
    Case64* C = P.cases + w.c;
    State64* st = P.state + w.c;
    const int s = w.s;
    const Species64& S = C->sp[s];
    const int N = C->n_cells;
    const bool periodic = C->bc == 1;
    const bool implicit = C->scheme == 1;
    const uint32_t step32 = (uint32_t)st->step_push;
    const uint32_t k0 = C->key0, k1 = C->key1;
    const int n = st->n_cur[s];
    int chunk = (n + w.nb - 1) / w.nb;
    chunk = (chunk + 63) & ~63;
    const int start = w.b * chunk, end = min(n, start + chunk);
    double ad[A_ND];
    unsigned ac[C_NU];
    for (int k = 0; k < A_ND; ++k) ad[k] = 0.0;
    for (int k = 0; k < C_NU; ++k) ac[k] = 0u;
    const double ku = S.kin_unit;
    for (int i = start + (int)threadIdx.x; i < end; i += kBlock) {
        if (!S.alive[i]) continue;
        double x = S.xi[i];
        const int j = (int)floor(x);
        double E;
        if (C->gather == 0) {
            E = C->E[j];
        } else {
            auto node = [&](int g) -> double {
                if (periodic) return 0.5 * (C->E[(g - 1 + N) % N] + C->E[g % N]);
                if (g == 0) return C->E[0];
                if (g == N) return C->E[N - 1];
                return 0.5 * (C->E[g - 1] + C->E[g]);
            };
            const double f = x - j;
            E = (1.0 - f) * node(j) + f * node(j + 1);
        }
        double vy = S.vy[i], vz = S.vz[i];
        double vold, vx, ab = 0.0;
        if (implicit) {
            // stored x~, v~ = v_{n-1/2} + abar/2; a at x~
            const double a = S.accel * E;
            ab = S.abar[i];
            vold = S.vx[i] - 0.5 * ab;
            vx = S.vx[i] + 0.5 * a;
            x += 0.5 * a;
            ab = 0.5 * (ab + a);
        } else {
            vold = S.vx[i];
            vx = vold + S.accel * E;
            x += vx;
        }
        ad[A_WORK] += ku * (vx - vold) * (vx + vold);
        bool absorbed;
        renorm64(x, N, periodic, absorbed);
        if (absorbed) {
            const int e = (x < 0.0) ? 0 : 1;
            ad[A_ABS0 + e] += ku * (vx * vx + vy * vy + vz * vz);
            ac[C_ABS0 + e] += 1u;
            S.alive[i] = 0;
            continue;
        }
        if (C->collisions && S.n_proc > 0) {
            const uint64_t id = S.id[i];
            // null-collision candidacy by waiting time (count, capped flag)
            const uint32_t wt = S.wait[i];
            const uint32_t cnt = wt & PIC_WAIT_MAX;
            bool cand = false;
            if (cnt > 0) {
                S.wait[i] = (cnt - 1) | (wt & PIC_WAIT_CAPPED);
            } else {
                cand = true;
                if (wt & PIC_WAIT_CAPPED) {
                    const uint4 r4 = philox((uint32_t)id, (uint32_t)(id >> 32), step32,
                                            ((uint32_t)s << 28) | 4u, k0, k1);
                    const double W = floor(log(u01d(r4.x)) * S.inv_log1mp);
                    if (W >= 1.0) {
                        cand = false;
                        const double Wm = W - 1.0;
                        S.wait[i] = Wm > (double)PIC_WAIT_MAX ? (PIC_WAIT_MAX | PIC_WAIT_CAPPED)
                                                              : (uint32_t)Wm;
                    }
                }
            }
            if (cand) {
                const uint4 r0 = philox((uint32_t)id, (uint32_t)(id >> 32), step32,
                                        (uint32_t)s << 28, k0, k1);
                S.wait[i] = geo_wait64(r0.x, S.inv_log1mp);
                ac[C_CAND] += 1u;
                const double k_in = ku * (vx * vx + vy * vy + vz * vz);
                const double u1 = u01d(r0.y);
                int kind = -1;
                if (s == 0) {
                    const double v2 = vx * vx + vy * vy + vz * vz, vm = sqrt(v2);
                    double t = v2 * S.t_scale + S.t_off;
                    if (t > S.t_max) ac[C_OVER] += 1u;
                    t = fmin(fmax(t, 0.0), S.t_max);
                    const int k = min((int)t, (int)S.t_max - 1);
                    const double f = t - k;
                    double cum = 0.0;
                    int slot = -1;
                    for (int p = 0; p < S.n_proc && slot < 0; ++p) {
                        const double sg = v2 > S.thr_v2[p]
                                              ? (1.0 - f) * S.tab[4 * k + p] + f * S.tab[4 * k + 4 + p]
                                              : 0.0;
                        cum += sg * vm;
                        if (u1 < cum) slot = p;
                    }
                    if (slot >= 0) {
                        kind = S.kind[slot];
                        double dx, dy, dz;
                        iso_dir64(u01d(r0.z), u01d(r0.w), dx, dy, dz);
                        if (kind == PIC_ELASTIC) {
                            const double cchi = vm > 0 ? (vx * dx + vy * dy + vz * dz) / vm : 0.0;
                            const double sp = sqrt(v2 * (1.0 - S.recoil2 * (1.0 - cchi)));
                            vx = sp * dx; vy = sp * dy; vz = sp * dz;
                        } else if (kind == PIC_EXCITATION) {
                            const double sp = sqrt(fmax(v2 - S.thr_v2[slot], 0.0));
                            vx = sp * dx; vy = sp * dy; vz = sp * dz;
                        } else {
                            const uint4 r1 = philox((uint32_t)id, (uint32_t)(id >> 32), step32, 1u, k0, k1);
                            const uint4 r3 = philox((uint32_t)id, (uint32_t)(id >> 32), step32, 3u, k0, k1);
                            const double B = S.opal_B;
                            const double avail = fmax(v2 - S.thr_v2[slot], 0.0) * S.eps_unit;
                            const double eej = B * tan(u01d(r1.x) * atan(avail / (2.0 * B)));
                            const double esc = fmax(avail - eej, 0.0);
                            const double s1 = sqrt(esc / S.eps_unit);
                            vx = s1 * dx; vy = s1 * dy; vz = s1 * dz;
                            double ex, ey, ez;
                            iso_dir64(u01d(r1.y), u01d(r1.z), ex, ey, ez);
                            const double s2 = sqrt(eej / S.eps_unit);
                            double n1, n2, n3, n4;
                            box_muller64(u01d(r3.x), u01d(r3.y), n1, n2);
                            box_muller64(u01d(r3.z), u01d(r3.w), n3, n4);
                            const double vt = C->sp[0].vth_newion;
                            append64(C, st, 0, s, x, s2 * ex, s2 * ey, s2 * ez,
                                     child_id(id, step32, 0u, k0, k1), step32, k0, k1, ad, ac);
                            append64(C, st, 1, s, x, vt * n1, vt * n2, vt * n3,
                                     child_id(id, step32, 1u, k0, k1), step32, k0, k1, ad, ac);
                        }
                    }
                } else {
                    const uint4 r2 = philox((uint32_t)id, (uint32_t)(id >> 32), step32,
                                            (1u << 28) | 2u, k0, k1);
                    double n1, n2, n3, n4;
                    box_muller64(u01d(r2.x), u01d(r2.y), n1, n2);
                    box_muller64(u01d(r2.z), u01d(r2.w), n3, n4);
                    const double wx = S.vth_neutral * n1, wy = S.vth_neutral * n2,
                                 wz = S.vth_neutral * n3;
                    const double gx = vx - wx, gy = vy - wy, gz = vz - wz;
                    const double g2 = gx * gx + gy * gy + gz * gz;
                    double t = g2 * S.t_scale + S.t_off;
                    if (t > S.t_max) ac[C_OVER] += 1u;
                    t = fmin(fmax(t, 0.0), S.t_max);
                    const int k = min((int)t, (int)S.t_max - 1);
                    const double f = t - k;
                    const double sg = (1.0 - f) * S.tab[k] + f * S.tab[k + 1];
                    if (u1 < sg * sqrt(g2)) {
                        kind = PIC_CHARGE_EXCHANGE;
                        vx = wx; vy = wy; vz = wz;
                    }
                }
                if (kind >= 0) {
                    ac[C_COLL0 + kind] += 1u;
                    ad[A_COLL] += ku * (vx * vx + vy * vy + vz * vz) - k_in;
                    S.vy[i] = vy;
                    S.vz[i] = vz;
                }
            }
        }
        // kinetic energy at n+1/2
        const double kh = ku * (vx * vx + vy * vy + vz * vz);
        ad[A_KAFT] += kh;
        if (implicit) {
            // predict the next step: v~ = v + abar/2, x~ = x + v~
            const double vt = vx + 0.5 * ab;
            x += vt;
            renorm64(x, N, periodic, absorbed);
            if (absorbed) {
                const int e = (x < 0.0) ? 0 : 1;
                ad[A_KAFT] -= kh;
                ad[A_ABS0 + e] += kh;
                ac[C_ABS0 + e] += 1u;
                S.alive[i] = 0;
                continue;
            }
            S.abar[i] = ab;
            vx = vt;
        }
        S.xi[i] = x;
        S.vx[i] = vx;
    }
    // the workgroup's ledger terms, one atomic each
    __shared__ double sd[kWaves][A_ND];
    __shared__ unsigned su[kWaves][C_NU];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < A_ND; ++k) {
        const double v = wave_sum(ad[k]);
        if (lane == 0) sd[wave][k] = v;
    }
    for (int k = 0; k < C_NU; ++k) {
        const unsigned v = wave_sum(ac[k]);
        if (lane == 0) su[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[A_ND];
        unsigned long long u[C_NU];
        for (int k = 0; k < A_ND; ++k) {
            t[k] = 0.0;
            for (int q = 0; q < kWaves; ++q) t[k] += sd[q][k];
        }
        for (int k = 0; k < C_NU; ++k) {
            u[k] = 0ull;
            for (int q = 0; q < kWaves; ++q) u[k] += su[q][k];
        }
        Led64& L = st->led;
        const int o = 1 - s;
        atomicAdd(&L.work[s], t[A_WORK]);
        atomicAdd(&L.K_after[s], t[A_KAFT]);
        atomicAdd(&L.coll[s], t[A_COLL]);
        atomicAdd(&L.absK[s][0], t[A_ABS0]);
        atomicAdd(&L.absK[s][1], t[A_ABS1]);
        if (t[A_COLL_O] != 0.0) atomicAdd(&L.coll[o], t[A_COLL_O]);
        if (t[A_KAFT_O] != 0.0) atomicAdd(&L.K_after[o], t[A_KAFT_O]);
        if (t[A_ABS0_O] != 0.0) atomicAdd(&L.absK[o][0], t[A_ABS0_O]);
        if (t[A_ABS1_O] != 0.0) atomicAdd(&L.absK[o][1], t[A_ABS1_O]);
        atomicAdd(&L.abs_n[s][0], u[C_ABS0]);
        atomicAdd(&L.abs_n[s][1], u[C_ABS1]);
        for (int k = 0; k < 4; ++k)
            if (u[C_COLL0 + k]) atomicAdd(&L.n_coll[s][k], u[C_COLL0 + k]);
        atomicAdd(&L.n_cand[s], u[C_CAND]);
        if (u[C_CRE0]) atomicAdd(&L.n_created[0], u[C_CRE0]);
        if (u[C_CRE1]) atomicAdd(&L.n_created[1], u[C_CRE1]);
        if (u[C_ABS0_O]) atomicAdd(&L.abs_n[o][0], u[C_ABS0_O]);
        if (u[C_ABS1_O]) atomicAdd(&L.abs_n[o][1], u[C_ABS1_O]);
        if (u[C_OVER]) atomicAdd(&L.n_over[s], u[C_OVER]);
    }
}

}  // namespace pic

using namespace pic;

namespace {

constexpr double QE = 1.602176634e-19;
constexpr double KB = 1.380649e-23;

struct Ref64 {
    std::vector<void*> allocs;
    std::vector<Case64> cases_h;
    Case64* d_cases = nullptr;
    State64* d_state = nullptr;
    Work* d_work = nullptr;
    std::vector<Work> work;
    int maxN = 0;
};

}  // namespace

// Accessors into the main context (pic_runtime.hip).
// Internal accessors into the main context (defined in pic_runtime.hip): the
// device case table read back to the host, the stream, the FP64-form slot,
// per-case configuration, table scale n_g (dx/dt)/nu_max and capacities, and
// the context's float64 copy of the input cross sections.
extern "C" int pic__ctx_export(pic_ctx* ctx, void** cases_h_out, int* n_cases,
                               hipStream_t* stream, void*** fp64_slot);
extern "C" int pic__ctx_case_info(pic_ctx* ctx, int32_t case_id, pic_case_config* cfg,
                                  double* scale, int64_t* cap);
extern "C" int pic__ctx_table(pic_ctx* ctx, int32_t s, int32_t p, int32_t* n,
                              const double** sigma);
extern "C" void** pic__ctx_fp64_slot(pic_ctx* ctx);
extern "C" int pic__ctx_species_consts(pic_ctx* ctx, int32_t k, int32_t s, double* out12);

extern "C" void pic__fp64_free(pic_ctx* ctx)
{
    void** slot = ctx ? pic__ctx_fp64_slot(ctx) : nullptr;
    if (!slot || !*slot) return;
    Ref64* r = (Ref64*)*slot;
    for (void* p : r->allocs) (void)hipFree(p);
    delete r;
    *slot = nullptr;
}

namespace {

template <typename T>
int alloc64(Ref64* r, T** p, size_t n)
{
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return PIC_E_NOMEM;
    if (hipMemset(q, 0, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return PIC_E_DEVICE;
    r->allocs.push_back(q);
    *p = (T*)q;
    return PIC_OK;
}

}  // namespace

extern "C" int pic_fp64_reference_init(pic_ctx* ctx)
{
    if (!ctx) return PIC_E_INVAL;
    void** slot = nullptr;
    int nc = 0;
    hipStream_t stream;
    void* chv = nullptr;
    if (pic__ctx_export(ctx, &chv, &nc, &stream, &slot)) return PIC_E_STATE;
    pic__fp64_free(ctx);
    Ref64* r = new Ref64();
    *slot = r;
    const Case* cases = (const Case*)chv;
    pic_diag d;
    std::vector<State64> st(nc);
    std::memset(st.data(), 0, sizeof(State64) * nc);
    r->cases_h.resize(nc);
    const int tile = 8192;
    for (int k = 0; k < nc; ++k) {
        const Case& C = cases[k];
        pic_case_config cfg;
        double scale[2];
        int64_t cap[2];
        if (pic__ctx_case_info(ctx, k, &cfg, scale, cap)) return PIC_E_STATE;
        // the plain form has the m = 1 EC and the MC weighting on uniform grids,
        // explicit and D1 implicit, without subcycling
        if (cfg.gather == PIC_GATHER_EC2 || C.nonuniform || C.ion_sub > 1) return PIC_E_INVAL;
        Case64& D = r->cases_h[k];
        std::memset(&D, 0, sizeof(Case64));
        const int N = C.n_cells;
        r->maxN = std::max(r->maxN, N);
        D.n_cells = N;
        D.bc = C.bc;
        D.gather = C.gather;
        D.collisions = C.collisions;
        D.scheme = cfg.scheme;
        D.dx = C.dx;
        D.dt = C.dt;
        D.rf_volts = C.rf_volts;
        D.rf_omega = C.rf_omega;
        D.background_rho = C.background_rho;
        D.key0 = C.key0;
        D.key1 = C.key1;
        if (alloc64(r, &D.Q[0], N + 1) || alloc64(r, &D.Q[1], N + 1) || alloc64(r, &D.E, N) ||
            alloc64(r, &D.phi, N + 1) || alloc64(r, &D.cnt[0], N) || alloc64(r, &D.cnt[1], N))
            return PIC_E_NOMEM;
        // particle state: the context's current live particles, widened
        std::memset(&d, 0, sizeof(d));
        if (pic_diagnostics(ctx, k, 0, &d)) return PIC_E_STATE;
        std::vector<int32_t> cell[2];
        std::vector<float> off[2], vx[2], vy[2], vz[2], ab[2];
        std::vector<uint64_t> idv[2];
        std::vector<uint32_t> wtv[2];
        pic_diag e;
        std::memset(&e, 0, sizeof(e));
        for (int s = 0; s < 2; ++s) {
            const size_t n = (size_t)d.n_slots[s];
            cell[s].resize(n); off[s].resize(n); vx[s].resize(n); vy[s].resize(n);
            vz[s].resize(n); ab[s].resize(n); idv[s].resize(n); wtv[s].resize(n);
            e.state_cap[s] = (int64_t)n;
            e.cell[s] = cell[s].data(); e.off[s] = off[s].data(); e.vx[s] = vx[s].data();
            e.vy[s] = vy[s].data(); e.vz[s] = vz[s].data(); e.id[s] = idv[s].data();
            e.abar[s] = ab[s].data();
            e.mcc_wait[s] = wtv[s].data();
        }
        if (pic_diagnostics(ctx, k, PIC_DIAG_STATE, &e)) return PIC_E_STATE;
        for (int s = 0; s < 2; ++s) {
            Species64& S = D.sp[s];
            const Species& F = C.sp[s];
            S.capacity = cap[s];
            S.accel = F.accel;
            S.qw_dx = F.qw_dx;
            S.kin_unit = F.kin_unit;
            S.chi_coef = F.chi_coef;
            double c64[12];
            if (pic__ctx_species_consts(ctx, k, s, c64)) return PIC_E_STATE;
            S.eps_unit = c64[0];
            S.opal_B = c64[1];
            S.recoil2 = c64[2];
            S.vth_neutral = c64[3];
            S.vth_newion = c64[4];
            S.t_scale = c64[5];
            S.t_off = c64[6];
            S.t_max = c64[7];
            for (int p = 0; p < kMaxProc; ++p) {
                S.thr_v2[p] = c64[8 + p];
                S.kind[p] = F.kind[p];
            }
            S.n_proc = F.n_proc;
            S.cand_thr = F.cand_thr;
            S.inv_log1mp = F.inv_log1mp;
            // float64 tables from the context's copy of the input cross sections
            if (S.n_proc > 0) {
                const int n = (int)F.t_max + 1;
                const int w = s == 0 ? 4 : 1;
                std::vector<double> td((size_t)n * w, 0.0);
                for (int p = 0; p < S.n_proc; ++p) {
                    const double* sig = nullptr;
                    int32_t nn = 0;
                    if (pic__ctx_table(ctx, s, p, &nn, &sig) || nn != n) return PIC_E_STATE;
                    for (int i = 0; i < n; ++i) td[(size_t)i * w + p] = sig[i] * scale[s];
                }
                double* dt = nullptr;
                if (alloc64(r, &dt, td.size())) return PIC_E_NOMEM;
                if (hipMemcpy(dt, td.data(), 8 * td.size(), hipMemcpyHostToDevice) != hipSuccess)
                    return PIC_E_DEVICE;
                S.tab = dt;
            }
            const size_t c = (size_t)cap[s];
            if (alloc64(r, &S.xi, c) || alloc64(r, &S.vx, c) || alloc64(r, &S.vy, c) ||
                alloc64(r, &S.vz, c) || alloc64(r, &S.abar, c) || alloc64(r, &S.id, c) ||
                alloc64(r, &S.alive, c) || alloc64(r, &S.wait, c))
                return PIC_E_NOMEM;
            const int64_t live = e.n_particles[s];
            std::vector<double> xd(live), vxd(live), vyd(live), vzd(live), abd(live);
            std::vector<int32_t> al(live, 1);
            double K = 0.0;
            for (int64_t i = 0; i < live; ++i) {
                xd[i] = (double)cell[s][i] + (double)off[s][i];
                vxd[i] = vx[s][i];
                vyd[i] = vy[s][i];
                vzd[i] = vz[s][i];
                abd[i] = cfg.scheme == PIC_IMPLICIT_D1 ? (double)ab[s][i] : 0.0;
                // v_{n-1/2}: the implicit state holds v~ = v_{n-1/2} + abar/2
                const double vh = vxd[i] - 0.5 * abd[i];
                K += F.kin_unit * (vh * vh + vyd[i] * vyd[i] + vzd[i] * vzd[i]);
            }
            st[k].led.K_after[s] = K;   // the kinetic energy the first step starts from
            if (live > 0) {
                if (hipMemcpy(S.xi, xd.data(), 8 * live, hipMemcpyHostToDevice) ||
                    hipMemcpy(S.vx, vxd.data(), 8 * live, hipMemcpyHostToDevice) ||
                    hipMemcpy(S.vy, vyd.data(), 8 * live, hipMemcpyHostToDevice) ||
                    hipMemcpy(S.vz, vzd.data(), 8 * live, hipMemcpyHostToDevice) ||
                    hipMemcpy(S.abar, abd.data(), 8 * live, hipMemcpyHostToDevice) ||
                    hipMemcpy(S.id, idv[s].data(), 8 * live, hipMemcpyHostToDevice) ||
                    hipMemcpy(S.alive, al.data(), 4 * live, hipMemcpyHostToDevice) ||
                    hipMemcpy(S.wait, wtv[s].data(), 4 * live, hipMemcpyHostToDevice))
                    return PIC_E_DEVICE;
            }
            st[k].n_next[s] = (int32_t)live;
            st[k].n_cur[s] = (int32_t)live;
            const int nb = (int)std::max<int64_t>(1, (cap[s] + tile - 1) / tile);
            for (int b = 0; b < nb; ++b) r->work.push_back(Work{k, s, b, nb});
        }
        st[k].step = d.step;
    }
    if (alloc64(r, &r->d_cases, nc) || alloc64(r, &r->d_state, nc) ||
        alloc64(r, &r->d_work, r->work.size()))
        return PIC_E_NOMEM;
    if (hipMemcpy(r->d_cases, r->cases_h.data(), sizeof(Case64) * nc, hipMemcpyHostToDevice) ||
        hipMemcpy(r->d_state, st.data(), sizeof(State64) * nc, hipMemcpyHostToDevice) ||
        hipMemcpy(r->d_work, r->work.data(), sizeof(Work) * r->work.size(), hipMemcpyHostToDevice))
        return PIC_E_DEVICE;
    return PIC_OK;
}

extern "C" int pic_fp64_reference_step(pic_ctx* ctx, int64_t n_steps)
{
    if (!ctx || n_steps < 0) return PIC_E_INVAL;
    void** slot = nullptr;
    int nc = 0;
    hipStream_t stream;
    void* chv = nullptr;
    if (pic__ctx_export(ctx, &chv, &nc, &stream, &slot) || !slot || !*slot)
        return PIC_E_STATE;
    Ref64* r = (Ref64*)*slot;
    Params64 p{r->d_cases, r->d_state, r->d_work};
    const int nb = (int)r->work.size();
    for (int64_t it = 0; it < n_steps; ++it) {
        hipLaunchKernelGGL(k64_deposit, dim3(nb), dim3(kBlock), 0, stream, p);
        hipLaunchKernelGGL(k64_solve, dim3(nc), dim3(kBlock), 8 * (2 * (size_t)r->maxN + 1),
                           stream, p);
        hipLaunchKernelGGL(k64_push, dim3(nb), dim3(kBlock), 0, stream, p);
    }
    if (hipGetLastError() != hipSuccess) return PIC_E_DEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return PIC_E_DEVICE;
    return PIC_OK;
}

extern "C" int pic_fp64_reference_state(pic_ctx* ctx, int32_t case_id, int32_t s, int64_t cap,
                                        double* xi, double* vx, double* vy, double* vz,
                                        double* abar, uint64_t* id, int64_t* n_out)
{
    if (!ctx || s < 0 || s > 1) return PIC_E_INVAL;
    void** slot = nullptr;
    int nc = 0;
    hipStream_t stream;
    void* chv = nullptr;
    if (pic__ctx_export(ctx, &chv, &nc, &stream, &slot) || !slot || !*slot)
        return PIC_E_STATE;
    if (case_id < 0 || case_id >= nc) return PIC_E_INVAL;
    Ref64* r = (Ref64*)*slot;
    if (hipStreamSynchronize(stream) != hipSuccess) return PIC_E_DEVICE;
    State64 st;
    if (hipMemcpy(&st, r->d_state + case_id, sizeof(State64), hipMemcpyDeviceToHost))
        return PIC_E_DEVICE;
    const Species64& S = r->cases_h[case_id].sp[s];
    const size_t n = (size_t)st.n_next[s];
    std::vector<double> a(n), b(n), c(n), e(n), f(n);
    std::vector<uint64_t> ii(n);
    std::vector<int32_t> al(n);
    if (n && (hipMemcpy(a.data(), S.xi, 8 * n, hipMemcpyDeviceToHost) ||
              hipMemcpy(b.data(), S.vx, 8 * n, hipMemcpyDeviceToHost) ||
              hipMemcpy(c.data(), S.vy, 8 * n, hipMemcpyDeviceToHost) ||
              hipMemcpy(e.data(), S.vz, 8 * n, hipMemcpyDeviceToHost) ||
              hipMemcpy(f.data(), S.abar, 8 * n, hipMemcpyDeviceToHost) ||
              hipMemcpy(ii.data(), S.id, 8 * n, hipMemcpyDeviceToHost) ||
              hipMemcpy(al.data(), S.alive, 4 * n, hipMemcpyDeviceToHost)))
        return PIC_E_DEVICE;
    int64_t k = 0;
    for (size_t i = 0; i < n; ++i) {
        if (!al[i]) continue;
        if (k < cap) {
            if (xi) xi[k] = a[i];
            if (vx) vx[k] = b[i];
            if (vy) vy[k] = c[i];
            if (vz) vz[k] = e[i];
            if (abar) abar[k] = f[i];
            if (id) id[k] = ii[i];
        }
        ++k;
    }
    if (n_out) *n_out = k;
    return k > cap ? PIC_E_CAPACITY : PIC_OK;
}

extern "C" int pic_fp64_reference_ledger(pic_ctx* ctx, int32_t case_id, pic_ledger* out)
{
    if (!ctx || !out) return PIC_E_INVAL;
    void** slot = nullptr;
    int nc = 0;
    hipStream_t stream;
    void* chv = nullptr;
    if (pic__ctx_export(ctx, &chv, &nc, &stream, &slot) || !slot || !*slot)
        return PIC_E_STATE;
    if (case_id < 0 || case_id >= nc) return PIC_E_INVAL;
    Ref64* r = (Ref64*)*slot;
    if (hipStreamSynchronize(stream) != hipSuccess) return PIC_E_DEVICE;
    State64 st;
    if (hipMemcpy(&st, r->d_state + case_id, sizeof(State64), hipMemcpyDeviceToHost))
        return PIC_E_DEVICE;
    const Led64& L = st.led;
    std::memset(out, 0, sizeof(pic_ledger));
    out->step = st.step_push;
    out->WE = L.WE;
    for (int s = 0; s < 2; ++s) {
        out->K_before[s] = L.K_before[s];
        out->K_after[s] = L.K_after[s];
        out->work[s] = L.work[s];
        out->coll_dK[s] = L.coll[s];
        for (int e = 0; e < 2; ++e) {
            out->absorbed_K[s][e] = L.absK[s][e];
            out->absorbed_n[s][e] = (int64_t)L.abs_n[s][e];
        }
        for (int k = 0; k < 4; ++k) out->n_coll[s][k] = (int64_t)L.n_coll[s][k];
        out->n_candidates[s] = (int64_t)L.n_cand[s];
        out->n_created[s] = (int64_t)L.n_created[s];
        out->n_over_table[s] = (int64_t)L.n_over[s];
        out->n_lost[s] = st.lost[s];
    }
    return PIC_OK;
}
