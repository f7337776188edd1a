// HIP kernels of the grid side of a step for gfx950 (MI355X): k_finalize
// (the FP64 field solve of the next step, Sec. II, and the energy ledger of
// the step just taken, one workgroup each per case), the compaction and sort
// of the particle arrays, and the set-up kernels (unit conversion, D1
// start-up, first waits, first deposit and solve).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"
#include "pic_common.hpp"
#include "pic_device.hpp"
#include "pic_weights.hpp"

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
// modified solve of the direct-implicit cycle (with m = 2: from the words of
// the dual grid, the row sums of the linearised deposit-gather operator).
// On a nonuniform grid the node charges are per unit area (rho times the
// node's volume), and the cell widths w_j enter the potential condition
// sum_j E_{j+1/2} w_j, the susceptibility (1/w_j) and the field energy.
// O(log N) deep.
// ---------------------------------------------------------------------------
constexpr double kEps0 = 8.8541878128e-12;

// ---------------------------------------------------------------------------
// Block-wide exclusive scans of small summaries (structs of doubles) in the
// order of the threads, or in the reverse order: comb(a, b) is "a, then b".
// Lanes combine by shuffles, wavefronts through LDS (wtot: kWv entries).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T shfl_T(const T& v, int d, bool down)
{
    T r;
    const double* s = (const double*)&v;
    double* o = (double*)&r;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 8); ++i)
        o[i] = down ? __shfl_down(s[i], d, 64) : __shfl_up(s[i], d, 64);
    return r;
}

template <int NT, typename T, typename Comb>
__device__ __forceinline__ T block_exscan(const T& x, const T& ident, Comb comb, bool rev,
                                          T* wtot)
{
    constexpr int kWv = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int pl = rev ? 63 - lane : lane;       // position in the scan order
    const int pw = rev ? kWv - 1 - wave : wave;
    T inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T prev = shfl_T(inc, o, rev);
        if (pl >= o) inc = comb(prev, inc);
    }
    T ex = shfl_T(inc, 1, rev);
    if (pl == 0) ex = ident;
    if (pl == 63) wtot[pw] = inc;
    lds_barrier();
    T pre = ident;
#pragma unroll
    for (int w = 0; w < kWv; ++w)
        if (w < pw) pre = comb(pre, wtot[w]);
    const T res = comb(pre, ex);
    lds_barrier();   // wtot may be written again
    return res;
}

struct Sum1 { double s; };
struct Proj2 { double m00, m01, m10, m11; };   // a 2x2 matrix up to a factor
template <int NR> struct Aff { double A; double B[NR]; };   // y -> A y + B (NR maps)

// ---------------------------------------------------------------------------
// Field solve with the tridiagonal m = 2 susceptibility (direct-implicit
// scheme): eps0 (1 + X) E = D0 + R, R_j = sum_{k<=j} sigma_k, X_jj = xd[j],
// X_{j,j+1} = X_{j+1,j} = xo[j] (xo[N-1]: the wrap, periodic only); D0 from
// dx sum_j E_j = phi_0 - phi_N.  (1 + X) u = 1 and (1 + X) v = R / eps0 by
// Gaussian elimination without pivoting (1 + X is symmetric positive
// definite: X is a sum of outer products of the particles' S_1 weights) in
// scans: the pivots by a scan of 2x2 matrices (c'_j = c_j / (b_j - a_j
// c'_{j-1}) is a continued fraction, i.e. a product of matrices up to a
// factor), the eliminated right-hand sides by an affine scan, the back
// substitution E_j = d'_j - c'_j E_{j+1} by an affine scan in reverse.  A
// periodic box takes the wrap coupling by Sherman-Morrison (a third
// right-hand side).  Thread t owns the Kr cells [t Kr, t Kr + Kr).  On a
// nonuniform grid (wr: w_j / dx, electrodes only) the operator acts on
// F_j = r_j E_j: (1/r + X) F = (D0 + R) / eps0, dx sum_j F_j = phi_0 - phi_N.
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void tridiag_field(const Case& Cc, State* st, long long next_step,
                                              long long field_step, bool sample_density,
                                              const double* S, const double* xd,
                                              const double* xo, double* red,
                                              const PIC_GLOBAL double* wr)
{
    constexpr int kRows = (PIC_MAX_CELLS + NT - 1) / NT;
    constexpr int NR = 3;   // right-hand sides: 1, R / eps0, the periodic correction
    const int N = Cc.n_cells, tid = threadIdx.x;
    const bool periodic = Cc.bc == 1;
    const double dx = Cc.dx;
    const int Kr = (N + NT - 1) / NT;
    const int j0 = tid * Kr;
    __shared__ double wbuf[(NT / 64) * 4];   // wave totals (up to 4 doubles each)
    __shared__ double ends[8];               // periodic: the solutions at rows 0 and N-1

    // Sherman-Morrison for the wrap: 1 + X = T + u v^T with u = (g, 0.., o),
    // v = (1, 0.., o / g), g = -(1 + xd_0); T loses the wrap coupling and
    // takes b_0 - g, b_{N-1} - o^2 / g
    const double o_w = periodic ? xo[N - 1] : 0.0;
    const double g_w = -((wr ? 1.0 / wr[0] : 1.0) + xd[0]);
    auto coef = [&](int j, double& a, double& b, double& c) {
        a = j > 0 ? xo[j - 1] : 0.0;
        c = j < N - 1 ? xo[j] : 0.0;
        b = (wr ? 1.0 / wr[j] : 1.0) + xd[j];
        if (periodic) {
            if (j == 0) b -= g_w;
            if (j == N - 1) b -= o_w * o_w / g_w;
        }
    };

    // R_j: prefix sums of the charges per area
    double sl = 0.0;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int j = j0 + k;
        if (k < Kr && j < N) sl += S[j];
    }
    const Sum1 rpre = block_exscan<NT>(Sum1{sl}, Sum1{0.0},
                                       [](const Sum1& x, const Sum1& y) { return Sum1{x.s + y.s}; },
                                       false, (Sum1*)wbuf);

    // pivots: (p, q) -> M_j (p, q), M_j = [[0, c_j], [-a_j, b_j]], c'_j = p / q
    auto pcomb = [](const Proj2& x, const Proj2& y) {
        // x, then y: the product y x, scaled
        Proj2 r{y.m00 * x.m00 + y.m01 * x.m10, y.m00 * x.m01 + y.m01 * x.m11,
                y.m10 * x.m00 + y.m11 * x.m10, y.m10 * x.m01 + y.m11 * x.m11};
        const double m = fmax(fmax(fabs(r.m00), fabs(r.m01)), fmax(fabs(r.m10), fabs(r.m11)));
        if (m > 0.0) {
            const double im = 1.0 / m;
            r.m00 *= im; r.m01 *= im; r.m10 *= im; r.m11 *= im;
        }
        return r;
    };
    Proj2 pl{1.0, 0.0, 0.0, 1.0};
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int j = j0 + k;
        if (k < Kr && j < N) {
            double a, b, c;
            coef(j, a, b, c);
            pl = pcomb(pl, Proj2{0.0, c, -a, b});
        }
    }
    const Proj2 ppre = block_exscan<NT>(pl, Proj2{1.0, 0.0, 0.0, 1.0}, pcomb, false,
                                        (Proj2*)wbuf);
    // c'_{j0 - 1} = (P (0, 1))_0 / (P (0, 1))_1
    double cprev = ppre.m01 / ppre.m11;
    if (j0 == 0) cprev = 0.0;

    // elimination: d'_j = alpha_j d'_{j-1} + beta_j, alpha_j = -a_j / den_j,
    // beta_j = r_j / den_j
    double cp[kRows], al[kRows], be[NR][kRows];
    Aff<NR> fl;
    fl.A = 1.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) fl.B[r] = 0.0;
    double R = rpre.s;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int j = j0 + k;
        cp[k] = 0.0;
        al[k] = 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r) be[r][k] = 0.0;
        if (k < Kr && j < N) {
            double a, b, c;
            coef(j, a, b, c);
            R += S[j];
            const double den = b - a * cprev;
            const double id = 1.0 / den;
            cp[k] = c * id;
            cprev = cp[k];
            al[k] = -a * id;
            be[0][k] = id;
            be[1][k] = R / kEps0 * id;
            be[2][k] = periodic ? (j == 0 ? g_w : (j == N - 1 ? o_w : 0.0)) * id : 0.0;
            fl.A *= al[k];
#pragma unroll
            for (int r = 0; r < NR; ++r) fl.B[r] = al[k] * fl.B[r] + be[r][k];
        }
    }
    auto acomb = [](const Aff<NR>& x, const Aff<NR>& y) {
        Aff<NR> r;
        r.A = y.A * x.A;
#pragma unroll
        for (int q = 0; q < NR; ++q) r.B[q] = y.A * x.B[q] + y.B[q];
        return r;
    };
    Aff<NR> idn;
    idn.A = 1.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) idn.B[r] = 0.0;
    const Aff<NR> fpre = block_exscan<NT>(fl, idn, acomb, false, (Aff<NR>*)wbuf);
    // d'_{j0 - 1} = fpre.B (d'_{-1} = 0); the eliminated right-hand sides
    {
        double dprev[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) dprev[r] = fpre.B[r];
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                be[r][k] = al[k] * dprev[r] + be[r][k];   // d'_j (rows past N: 0)
                if (k < Kr && j0 + k < N) dprev[r] = be[r][k];
            }
        }
    }
    // back substitution, last row first: E_j = -c'_j E_{j+1} + d'_j
    Aff<NR> bl = idn;
#pragma unroll
    for (int k = kRows - 1; k >= 0; --k) {
        if (k < Kr && j0 + k < N) {
            Aff<NR> rowm;
            rowm.A = -cp[k];
#pragma unroll
            for (int r = 0; r < NR; ++r) rowm.B[r] = be[r][k];
            bl = acomb(bl, rowm);
        }
    }
    const Aff<NR> bpre = block_exscan<NT>(bl, idn, acomb, true, (Aff<NR>*)wbuf);
    double y[NR][kRows];   // the solutions for the NR right-hand sides
    {
        double enext[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) enext[r] = bpre.B[r];   // E beyond the last row: 0
#pragma unroll
        for (int k = kRows - 1; k >= 0; --k) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                y[r][k] = 0.0;
                if (k < Kr && j0 + k < N) {
                    y[r][k] = be[r][k] - cp[k] * enext[r];
                    enext[r] = y[r][k];
                }
            }
        }
    }
    if (periodic) {
        // x = y - (v . y) / (1 + v . z) z for y = the solutions of 1 and R
        // (z: the third), v = (1, 0.., o / g)
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            const int j = j0 + k;
            if (k < Kr && (j == 0 || j == N - 1))
                for (int r = 0; r < NR; ++r) ends[(j == 0 ? 0 : 4) + r] = y[r][k];
        }
        lds_barrier();
        const double og = o_w / g_w;
        const double fac = 1.0 + ends[2] + og * ends[6];
        const double f0 = (ends[0] + og * ends[4]) / fac, f1 = (ends[1] + og * ends[5]) / fac;
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            y[0][k] -= f0 * y[2][k];
            y[1][k] -= f1 * y[2][k];
        }
    }
    // D0 / eps0 from dx sum E = phi_0 - phi_N: E = D0e u + v
    double su = 0.0, sv = 0.0;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        su += y[0][k];
        sv += y[1][k];
    }
    su = block_sum<double, NT>(su, red);
    sv = block_sum<double, NT>(sv, red);
    double V = 0.0;
    if (!periodic) {
        const double cyc = Cc.rf_freq * ((double)next_step * Cc.dt);
        V = Cc.rf_volts * sinpi(2.0 * (cyc - floor(cyc)));
    }
    const double D0e = (V / dx - sv) / su;
    // potentials: phi_{j+1} = phi_0 - dx sum_{k<=j} E_k
    double el = 0.0;
#pragma unroll
    for (int k = 0; k < kRows; ++k) el += D0e * y[0][k] + y[1][k];
    const Sum1 epre = block_exscan<NT>(Sum1{el}, Sum1{0.0},
                                       [](const Sum1& x, const Sum1& z) { return Sum1{x.s + z.s}; },
                                       false, (Sum1*)wbuf);
    const double phi0 = periodic ? 0.0 : V;
    if (tid == 0) gp(Cc.phi)[0] = phi0;
    double we = 0.0, run = epre.s;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int j = j0 + k;
        if (k < Kr && j < N) {
            const double F = D0e * y[0][k] + y[1][k];   // E; r E on a nonuniform grid
            const double r = wr ? wr[j] : 1.0;
            const double E = F / r;
            run += F;
            gp(Cc.E)[j] = E;
            gp(Cc.ehat[0])[j] = (float)(Cc.sp[0].accel * E);
            gp(Cc.ehat[1])[j] = (float)(Cc.sp[1].accel * E);
            gp(Cc.phi)[j + 1] = phi0 - dx * run;
            we += 0.5 * kEps0 * E * E * dx * r;
        }
    }
    we = block_sum<double, NT>(we, red);
    if (tid == 0) {
        st->WE[field_step & 1] = we;
        if (!isfinite(we)) atomicOr(&st->flags, 1);
        if (sample_density) st->dens_samples += 1;
    }
    lds_barrier();
}

// kDual: the code of the implicit m = 2 moment words is compiled in (the
// launches of batches without such a case leave it out: its registers would
// make the rest spill).  kPlain: every case has the EC gather (m = 1) on a
// uniform grid (no MC, m = 2 or nonuniform code).
template <int NT, bool kDual, bool kPlain = false>
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
    const bool node_chi = !kPlain && implicit && Cc.gather == 1;
    // node g = tid + k NT needs the counts and weights of cells g and g-1
    const PIC_GLOBAL unsigned long long* dc[2] = {gp((const unsigned long long*)Cc.dep_cnt[0]),
                                                  gp((const unsigned long long*)Cc.dep_cnt[1])};
    const PIC_GLOBAL unsigned long long* dw[2] = {gp((const unsigned long long*)Cc.dep_w[0]),
                                                  gp((const unsigned long long*)Cc.dep_w[1])};
    // Nodes in batches of kB per thread; inside a batch every load is issued
    // before any result is used (unconditional loads from clamped indices,
    // selected afterwards, so that none waits behind a branch).
    // (5 covers 2048 cells at NT = 512 in one batch; more than 1 with the
    // moment path would spill)
    constexpr int kB = kDual ? 1 : 5;
    const double qs0 = Cc.sp[0].qw_dx / kFixScale, qs1 = Cc.sp[1].qw_dx / kFixScale;
    // subcycled ions keep their deposit until the step in which they move
    // (and deposit again); they respond only to the field they are
    // corrected with, the one of the solve before that step (field_step:
    // the index of the step that uses this field; next_step is the time of
    // the boundary voltage, one later for the implicit field)
    const bool ions_move = Cc.ion_sub <= 1 || field_step % Cc.ion_sub == 0;
    const double chi0 = Cc.sp[0].chi_coef, chi1 = ions_move ? Cc.sp[1].chi_coef : 0.0;
    const double rho_bg = Cc.background_rho;
    const bool ec2 = !kPlain && Cc.gather == 2;   // quadratic deposit: node words
    const bool dual = kDual && implicit && ec2;   // moment words (deposit_moments)
    const bool nu = !kPlain && Cc.nonuniform != 0;
    const PIC_GLOBAL double* wjr = gp((const double*)Cc.cell_wr);   // nu: w_j / dx
    // m = 2 implicit: the second moment words (counts of the particles left
    // of their nearest node, sums of their weights to the node after it)
    const PIC_GLOBAL unsigned long long* dx_c[2] = {
        gp((const unsigned long long*)Cc.chi_cnt[0]), gp((const unsigned long long*)Cc.chi_cnt[1])};
    const PIC_GLOBAL unsigned long long* dx_w[2] = {
        gp((const unsigned long long*)Cc.chi_w[0]), gp((const unsigned long long*)Cc.chi_w[1])};
    // node g's outputs from its fixed-point charges q0, q1 and (g < N) the
    // particle counts c0, c1 of cell g
    auto emit_node = [&](int g, long long q0, long long q1, long long c0, long long c1) {
        double rho = rho_bg, chin = 0.0;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const long long q = s == 0 ? q0 : q1;
            gp(Cc.qfix[s])[g] = q;
            if (sample_density) gatomic_add(gp(&Cc.dens_acc[s][g]), (unsigned long long)q);
            rho += (double)q * (s == 0 ? qs0 : qs1);
            chin += (double)q * (s == 0 ? chi0 : chi1);
        }
        if (node_chi) {
            const bool end = !periodic && (g == 0 || g == N);
            if (nu) {
                // over the node's volume / dx: half of each adjacent cell
                const double vh = 0.5 * ((g > 0 ? wjr[g - 1] : 0.0) + (g < N ? wjr[g] : 0.0));
                Y[g] = chin / (kFixScale * vh);
            } else {
                Y[g] = chin * ((end ? 2.0 : 1.0) / kFixScale);
            }
        }
        double sg = rho * dx;
        if (nu) {
            // node volume / dx: half of each adjacent cell, the whole end cell
            const double vg =
                g == 0 ? wjr[0] : (g == N ? wjr[N - 1] : 0.5 * (wjr[g - 1] + wjr[g]));
            sg = (rho - rho_bg) * dx + rho_bg * dx * vg;
            rho = sg / (dx * vg);
        }
        gp(Cc.rho)[g] = rho;
        // R_j = sum_{k=1..j} (charge per area of node k): node 0's is zero
        S[g] = g == 0 ? 0.0 : sg;
        if (g < N) {
            gp(Cc.ccount[0])[g] = c0;
            gp(Cc.ccount[1])[g] = c1;
            if (!node_chi && !dual) {
                double chi = implicit ? chi0 * (double)c0 + chi1 * (double)c1 : 0.0;
                if (nu) chi /= wjr[g];
                X[g] = chi;
                // an explicit case's chi stays zero, as allocated (a case
                // keeps its scheme)
                if (implicit) gp(Cc.chi)[g] = chi;
            }
        }
    };
    if (dual) {
        // moment words (deposit_moments), one node at a time: counts and
        // weight sums of nodes g-1, g, g+1, folded at electrodes or wrapped
#pragma unroll 1
        for (int g = tid; g <= N; g += NT) {
            const int gg = (periodic && g == N) ? 0 : g;
            const int gp1 = periodic ? (gg + 1 == N ? 0 : gg + 1) : min(gg + 1, N);
            const int gm1 = periodic ? (gg > 0 ? gg - 1 : N - 1) : max(gg - 1, 0);
            long long q[2], nc[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const long long a0 = (long long)dw[s][gg], a1 = (long long)dw[s][gp1];
                const long long b0 = (long long)dx_w[s][gg], bm = (long long)dx_w[s][gm1];
                const long long n0 = (long long)dc[s][gg] + (long long)dx_c[s][gg];
                nc[s] = (long long)dc[s][gg] + (long long)dx_c[s][gp1];
                q[s] = n0 * (1ll << kFixBits) - a0 - b0;
                if (periodic) {
                    q[s] += a1 + bm;
                } else {
                    q[s] += gg < N ? a1 : b0;   // node N keeps its own P2 (folded)
                    q[s] += gg > 0 ? bm : a0;   // node 0 keeps its own P0 (folded)
                }
            }
            emit_node(g, q[0], q[1], nc[0], nc[1]);
        }
    } else {
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
            long long q[2];
#pragma unroll
            for (int s = 0; s < 2; ++s)
                q[s] = ec2 ? qn[k][s] : cn[k][s] * (1ll << kFixBits) - wr[k][s] + wl[k][s];
            emit_node(g, q[0], q[1], cn[k][0], cn[k][1]);
        }
    }
    }
    if (dual) {
        // Row sums of the susceptibility operator at the centres (the
        // diagonal approximation): the particles with nearest node e lie
        // between centres e-1 and e at fraction t towards e; centre h takes
        // sum (1 - t) of node h+1 and sum t of node h, i.e. n(h+1) 2^24 -
        // F(h+1) + F(h) with F(e) = sum t 2^24 = n(e) 2^23 + W2(e) - W0(e).
        // Next to an electrode the field beyond is zero and the centre takes
        // the square of its weight: F(0) = sum t^2 = 2 W2(0), and
        // n(N) 2^24 - F(N) = sum (1 - t)^2 = 2 W0(N).  Periodic: node N is 0.
        auto F = [&](int s, int e) -> long long {
            const long long n = (long long)dc[s][e] + (long long)dx_c[s][e];
            const long long a = (long long)dw[s][e], b = (long long)dx_w[s][e];
            if (!periodic && e == 0) return 2 * b;
            if (!periodic && e == N) return n * (1ll << kFixBits) - 2 * a;
            return n * (1ll << (kFixBits - 1)) + b - a;
        };
#pragma unroll 1
        for (int h = tid; h < N; h += NT) {
            {
                const int e1 = (periodic && h + 1 == N) ? 0 : h + 1;
                long long v[2];
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const long long n1 = (long long)dc[s][e1] + (long long)dx_c[s][e1];
                    v[s] = n1 * (1ll << kFixBits) - F(s, e1) + F(s, h);
                }
                const double chi = (chi0 * (double)v[0] + chi1 * (double)v[1]) / kFixScale;
                if (!nu) gp(Cc.chi)[h] = chi;   // the row sum of the operator
                // the operator itself: centre h takes (1 - t)^2 = 2 P0 from
                // the particles of node h + 1 and t^2 = 2 P2 from those of
                // node h; the particles of node h + 1 couple centres h and
                // h + 1 by t (1 - t) = 1/2 - P0 - P2 (none beyond an electrode).
                // On a nonuniform grid (electrodes only) each particle also
                // carries 1/r^2 of its cell: cell g - 1 for the particles left
                // of node g, cell g for those right of it.
                const bool couples = periodic || h + 1 < N;
                double dg = 0.0, cpl = 0.0;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const double cs = s == 0 ? chi0 : chi1;
                    if (!nu) {
                        dg += cs * (double)(2 * (long long)dx_w[s][h] + 2 * (long long)dw[s][e1]);
                        if (couples) {
                            const long long n1 = (long long)dc[s][e1] + (long long)dx_c[s][e1];
                            cpl += cs * (double)(n1 * (1ll << (kFixBits - 1)) -
                                                 (long long)dw[s][e1] - (long long)dx_w[s][e1]);
                        }
                    } else {
                        const PIC_GLOBAL unsigned long long* l0 = gp(Cc.chl_w0[s]);
                        const PIC_GLOBAL unsigned long long* l2 = gp(Cc.chl_w2[s]);
                        const double rh = wjr[h];
                        const double ih = 1.0 / (rh * rh);
                        const double il = h > 0 ? 1.0 / (wjr[h - 1] * wjr[h - 1]) : 0.0;
                        const double ir = h + 1 < N ? 1.0 / (wjr[h + 1] * wjr[h + 1]) : 0.0;
                        // node h: P2 of its left (cell h-1) and right (cell h) sides
                        const long long w2l = (long long)l2[h], w2 = (long long)dx_w[s][h];
                        // node h+1: P0 of its left (cell h) and right (cell h+1) sides
                        const long long w0l = (long long)l0[e1], w0 = (long long)dw[s][e1];
                        dg += cs * (2.0 * ((double)w2l * il + (double)(w2 - w2l) * ih) +
                                    2.0 * ((double)w0l * ih + (double)(w0 - w0l) * ir));
                        if (couples) {
                            const long long nl = (long long)dx_c[s][e1], nr = (long long)dc[s][e1];
                            const long long w2e = (long long)dx_w[s][e1], w2el = (long long)l2[e1];
                            const double left = (double)(nl * (1ll << (kFixBits - 1)) - w0l - w2el);
                            const double right =
                                (double)(nr * (1ll << (kFixBits - 1)) - (w0 - w0l) - (w2e - w2el));
                            cpl += cs * (left * ih + right * ir);
                        }
                    }
                }
                X[h] = dg / kFixScale;
                Y[h] = cpl / kFixScale;
            }
        }
    }
    lds_barrier();   // every deposit word has been read
    if (dual && nu) {
        // the response to a uniform field: chi_h = sum_h' X_hh' r_h'
        for (int h = tid; h < N; h += NT) {
            double x = X[h] * wjr[h];
            if (h > 0) x += Y[h - 1] * wjr[h - 1];
            if (h + 1 < N) x += Y[h] * wjr[h + 1];
            gp(Cc.chi)[h] = x;
        }
    }
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
            gp(Cc.dep_cnt[0])[j] = 0;
            gp(Cc.dep_w[0])[j] = 0;
            if (ions_move) {
                gp(Cc.dep_cnt[1])[j] = 0;
                gp(Cc.dep_w[1])[j] = 0;
            }
            if (dual) {
                gp(Cc.chi_cnt[0])[j] = 0;
                gp(Cc.chi_w[0])[j] = 0;
                if (nu) {
                    gp(Cc.chl_w0[0])[j] = 0;
                    gp(Cc.chl_w2[0])[j] = 0;
                }
                if (ions_move) {
                    gp(Cc.chi_cnt[1])[j] = 0;
                    gp(Cc.chi_w[1])[j] = 0;
                    if (nu) {
                        gp(Cc.chl_w0[1])[j] = 0;
                        gp(Cc.chl_w2[1])[j] = 0;
                    }
                }
            }
        }
    }
    if (dual) {
        // the m = 2 implicit field: the tridiagonal operator, solved as such
        tridiag_field<NT>(Cc, st, next_step, field_step, sample_density, S, X, Y, red,
                          nu ? wjr : nullptr);
        return;
    }
    // One pass of an associative scan gives every prefix the solve needs.
    // With sigma_j the charge per area of node j (sigma_0 = 0 stands for the
    // electrode or the periodic seam), kap_j = eps0 (1 + chi_j), om_j = w_j/dx
    // and c_j = om_j / kap_j, the running sums over cells k <= j are
    //   R_j = sum sigma_k,  B_j = sum c_k,  T_j = sum R_k c_k,
    // and then D_{j+1/2} = D0 + R_j, E_j = (D0 + R_j) / kap_j,
    // phi_{j+1} = phi_0 - dx (D0 B_j + T_j), with D0 fixed by
    // dx sum E_j om_j = phi_0 - phi_N: D0 = (V/dx - T_{N-1}) / B_{N-1}.
    // A run of cells summarises to (R, B, T); a run A followed by a run B
    // combines to (R_A + R_B, B_A + B_B, T_A + T_B + R_A B_B).  Thread t
    // takes the kPer cells [t kPer, t kPer + kPer) in order; lanes combine
    // by shuffles, wavefronts through LDS.
    constexpr int kWv = NT / 64;
    const int lane = tid & 63, wave = tid >> 6;
    const int Kr = (N + NT - 1) / NT;   // cells per thread (<= kPer, uniform)
    const int j0 = tid * Kr;
    // the thread's cells, read once and kept for the second pass: every
    // read of a cell is issued before the first is used
    double sj[kPer], kap[kPer], cj[kPer], omj[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (k < Kr) {
            const int j = min(j0 + k, N - 1);
            sj[k] = S[j];
            kap[k] = X[j];
            omj[k] = nu ? wjr[j] : 1.0;
        }
    }
    double rs = 0.0, bs = 0.0, ts = 0.0;   // this thread's run
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (k < Kr) {
            kap[k] = kEps0 * (1.0 + kap[k]);
            cj[k] = omj[k] / kap[k];
            if (j0 + k < N) {
                rs += sj[k];
                bs += cj[k];
                ts += rs * cj[k];
            }
        }
    }
    // inclusive scan over the lanes of the wavefront
    double ri = rs, bi = bs, ti = ts;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double rp = __shfl_up(ri, o, 64), bp = __shfl_up(bi, o, 64),
                     tp = __shfl_up(ti, o, 64);
        if (lane >= o) {
            ti = tp + ti + rp * bi;
            ri = rp + ri;
            bi = bp + bi;
        }
    }
    __shared__ double wtot[kWv][3];
    if (lane == 63) {
        wtot[wave][0] = ri;
        wtot[wave][1] = bi;
        wtot[wave][2] = ti;
    }
    // the lanes before this one (exclusive)
    double re = __shfl_up(ri, 1, 64), be = __shfl_up(bi, 1, 64), te = __shfl_up(ti, 1, 64);
    if (lane == 0) re = be = te = 0.0;
    lds_barrier();
    // the wavefronts before this one, then every wavefront (the totals)
    double rw = 0.0, bw = 0.0, tw = 0.0, rt = 0.0, bt = 0.0, tt = 0.0;
#pragma unroll
    for (int w = 0; w < kWv; ++w) {
        const double r2 = wtot[w][0], b2 = wtot[w][1], t2 = wtot[w][2];
        if (w < wave) {
            tw = tw + t2 + rw * b2;
            rw += r2;
            bw += b2;
        }
        tt = tt + t2 + rt * b2;
        rt += r2;
        bt += b2;
    }
    // this thread's starting prefix: the earlier wavefronts, then the
    // earlier lanes
    double R = rw + re, B = bw + be, T = tw + te + rw * be;
    double V = 0.0;
    if (!periodic) {
        // V0 sin(2 pi f t) through the phase in cycles reduced to [0, 1)
        const double cyc = Cc.rf_freq * ((double)next_step * Cc.dt);
        V = Cc.rf_volts * sinpi(2.0 * (cyc - floor(cyc)));
    }
    const double D0 = (V / dx - tt) / bt;
    const double phi0 = periodic ? 0.0 : V;
    if (tid == 0) gp(Cc.phi)[0] = phi0;
    // E_j and phi_{j+1} of the thread's cells are staged in LDS over S and X
    // (every read of those precedes the last barrier) and stored by
    // consecutive threads: one line per 16 lanes instead of one per 4
    double* Es = S;
    double* Ps = X;
    double we = 0.0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int j = j0 + k;
        if (k < Kr && j < N) {
            R += sj[k];
            B += cj[k];
            T += R * cj[k];
            const double E = (D0 + R) / kap[k];
            Es[j] = E;
            Ps[j] = phi0 - dx * (D0 * B + T);
            we += 0.5 * kEps0 * E * E * dx * omj[k];
        }
    }
    we = block_sum<double, NT>(we, red);   // its barriers publish Es and Ps
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int j = tid + k * NT;
        if (j < N) {
            const double E = Es[j];
            gp(Cc.E)[j] = E;
            gp(Cc.ehat[0])[j] = (float)(Cc.sp[0].accel * E);
            gp(Cc.ehat[1])[j] = (float)(Cc.sp[1].accel * E);
            gp(Cc.phi)[j + 1] = Ps[j];
        }
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
    // the workgroup partials with kU loads in flight (one pass covers 64 kU
    // rows), then a wavefront tree; the order of the sums is fixed
    constexpr int kU = 24;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const PIC_GLOBAL double* pd = gp(pd_);
    const PIC_GLOBAL unsigned* pu = gp(pu_);
    for (int f = wave; f < PD_N + PU_N; f += NT / 64) {
        if (f < PD_N) {
            double acc = 0.0;
            // unconditional loads from clamped indices keep all kU in flight
            const PIC_GLOBAL double* row = pd + (size_t)f * stride + fb;
            for (int b = lane; b < nb; b += 64 * kU) {
                double x[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) x[u] = row[min(b + 64 * u, nb - 1)];
#pragma unroll
                for (int u = 0; u < kU; ++u) acc += b + 64 * u < nb ? x[u] : 0.0;
            }
            const double v = wave_sum(acc);
            if (lane == 0) sd[f] = v;
        } else {
            // per-step counts of one case fit in 32 bits
            unsigned a = 0u;
            const PIC_GLOBAL unsigned* row = pu + (size_t)(f - PD_N) * stride + fb;
            for (int b = lane; b < nb; b += 64 * kU) {
                unsigned x[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) x[u] = row[min(b + 64 * u, nb - 1)];
#pragma unroll
                for (int u = 0; u < kU; ++u) a += b + 64 * u < nb ? x[u] : 0u;
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

// ---------------------------------------------------------------------------
// k_finalize: two workgroups per case (kFinStep threads) after the particle pass, running side
// by side: the odd one closes the ledger of the step (reduction of the
// workgroup partials), the even one solves the FP64 field of the next step.
// They write disjoint fields of the case state (flags through atomics).
// ---------------------------------------------------------------------------
template <bool kDual, bool kPlain>
__global__ __launch_bounds__(kFinStep) void k_finalize(Params P, int sample)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kFinStep / 64];
    __shared__ double sd[PD_N];
    __shared__ long long si[PU_N];
    Case* C = P.cases + (blockIdx.x >> 1);
    State* st = P.state + (blockIdx.x >> 1);
    // a launch for one scheme group (mode = its scheme; -1 = every case)
    if (P.mode >= 0 && C->scheme != P.mode) return;
    if (blockIdx.x & 1) {
        // ledger of the step just taken
        reduce_partials<kFinStep>(P.pd, P.pu, P.stride, C->first_block, C->n_blocks, sd, si);
        finish_ledger(C, st, sd, si);
        return;
    }
    // field of the next step (every thread reads st->step once; thread 0
    // writes it after the solve's last barrier).  A relaxed atomic load is
    // read exactly once without the wait a volatile load carries, so it
    // travels with the case's own loads.
    const long long next =
        __hip_atomic_load(&st->step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
    solve_case<kFinStep, kDual, kPlain>(C, st, next + (C->scheme == 1 ? 1 : 0), next,
                                        sample != 0, (double*)smem, red);
    if (threadIdx.x == 0) {
        if (sample) st->eedf_samples += 1;
        st->step = next;
    }
}
template __global__ void k_finalize<false, true>(Params, int);
template __global__ void k_finalize<false, false>(Params, int);
template __global__ void k_finalize<true, false>(Params, int);

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
    // the clock of the species' first move (drawn waits count from it)
    const uint32_t clk0 = clock_from(st->step, w.s == 1 ? C->ion_sub : 1,
                                     C->collisions && S.n_proc > 0);
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
            wt = wait_field(clk0, wait_encode(geo0(r4.x, S.inv_log1mp)));
        }
        float o = S.off[i];
        if (startup) {
            // the first prediction x~ = x + K v, K the species' step
            const float kf = w.s == 1 ? (float)C->ion_sub : 1.0f;
            S.abar[i] = 0.0f;
            if (C->nonuniform) {
                walk(c, o, kf * S.vx[i], C->cell_r, C->cell_run, N);
            } else {
                o += kf * S.vx[i];
                renorm(c, o);
            }
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
    for (int base = start; base < end; base += kBlock * kScatterILP) {
        int32_t cw[kScatterILP];
#pragma unroll
        for (int k = 0; k < kScatterILP; ++k)
            cw[k] = cellp[min(base + k * kBlock + (int)threadIdx.x, end - 1)];
#pragma unroll
        for (int k = 0; k < kScatterILP; ++k) {
            const int i = base + k * kBlock + (int)threadIdx.x;
            const int c = i < end ? cell_of(cw[k]) : -1;
            const int b = c >= 0 ? c >> sh : -1;
            wave_count_add(lh, b, b >= 0);
            if (b >= 0) range_note(lo, hi, b);
        }
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

// The scatter moves kScatterILP particles per thread at a time: their loads
// are issued together, then their slots are taken (LDS counters of the
// chunk's runs), then they are stored.
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
    const float hk = 0.5f * (w.s == 1 ? (float)C->ion_sub : 1.0f);   // K/2
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
    for (int base = start; base < end; base += kBlock * kScatterILP) {
        int32_t cw[kScatterILP];
#pragma unroll
        for (int k = 0; k < kScatterILP; ++k)
            cw[k] = cellp[min(base + k * kBlock + (int)threadIdx.x, end - 1)];
#pragma unroll
        for (int k = 0; k < kScatterILP; ++k) {
            const int i = base + k * kBlock + (int)threadIdx.x;
            const int c = i < end ? cell_of(cw[k]) : -1;
            const int b = c >= 0 ? c >> sh : -1;
            wave_count_add(lh, b, b >= 0);
            if (b >= 0) range_note(lo, hi, b);
        }
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
    for (int base = start; base < end; base += kBlock * kScatterILP) {
        int32_t w0[kScatterILP];
        float o[kScatterILP], vx[kScatterILP], ab[kScatterILP];
        u32x4 rc[kScatterILP];
#pragma unroll
        for (int k = 0; k < kScatterILP; ++k) {
            const int j = min(base + k * kBlock + (int)threadIdx.x, end - 1);
            w0[k] = cellp[j];
            o[k] = offp[j];
            vx[k] = vxp[j];
            rc[k] = recp[j];
            ab[k] = imp ? abp[j] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < kScatterILP; ++k) {
            const int i = base + k * kBlock + (int)threadIdx.x;
            const int c = i < end ? cell_of(w0[k]) : -1;
            const int b = c >= 0 ? c >> sh : -1;
            const unsigned r = wave_count_add(lh, b, b >= 0);
            if (c < 0) continue;
            const unsigned d = lb[b] + r;
            cell2[d] = w0[k];
            off2[d] = o[k];
            vx2[d] = vx[k];
            rec2[d] = rc[k];
            float vh = vx[k];
            if (imp) {
                ab2[d] = ab[k];
                vh = vx[k] - hk * ab[k];   // v_{n-1/2} from the stored prediction
            }
            const float vy = rec_vy(rc[k]), vz = rec_vz(rc[k]);
            v2 += (double)(vh * vh + vy * vy + vz * vz);
        }
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
    const bool ec2 = C->gather == 2, periodic = C->bc == 1;
    const bool dual = dual_chi(C->scheme, C->gather);
    unsigned long long* dep = (unsigned long long*)smem;
    unsigned long long* dch = dep + (N + 1);   // dual: susceptibility words
    // and on a nonuniform grid the left-side P0 and P2 sums
    const bool duo = dual && C->nonuniform;
    unsigned long long* dl0 = duo ? dch + (N + 1) : nullptr;
    unsigned long long* dl2 = duo ? dl0 + (N + 1) : nullptr;
    for (int j = threadIdx.x; j <= N; j += kBlock) {
        dep[j] = 0ull;
        if (dual) dch[j] = 0ull;
        if (duo) {
            dl0[j] = 0ull;
            dl2[j] = 0ull;
        }
    }
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
        if (dual) {
            deposit_moments(dep, dch, true, c, S.off[i], N, periodic, lo, hi, false, dl0, dl2);
        } else if (ec2) {
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
        const unsigned long long d = dual ? dch[j] : 0ull;
        if (d) {
            atomicAdd(&C->chi_cnt[w.s][j], d >> 40);
            atomicAdd(&C->chi_w[w.s][j], d & kWMask);
        }
        if (duo) {
            if (dl0[j]) atomicAdd(&C->chl_w0[w.s][j], dl0[j]);
            if (dl2[j]) atomicAdd(&C->chl_w2[w.s][j], dl2[j]);
        }
    }
}

__global__ __launch_bounds__(kFinBlock) void k_solve(Params P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kFinBlock / 64];
    Case* C = P.cases + blockIdx.x;
    State* st = P.state + blockIdx.x;
    solve_case<kFinBlock, true>(C, st, st->step + (C->scheme == 1 ? 1 : 0), st->step, false,
                          (double*)smem, red);
}

}  // namespace pic
