/*
 * FP64 CPU oracle for the EC electrostatic PIC/MCC step of arXiv:1310.5284.
 *
 * TEST INFRASTRUCTURE ONLY (see pic_oracle.h): loaded by the tests, the smoke
 * check and the CPU-baseline leg of the benchmark; never by the GPU library.
 *
 * What the paper fixes and where:
 *   - charge weighting with S_m at the nodes .................. Sec. II, Eq. (2)
 *   - field interpolation with S_{m-1} of the field at the
 *     half-grid points x_{g+1/2} ................................ Sec. II, Eq. (3)
 *   - the four schemes (MC/EC x explicit/direct-implicit) ....... Sec. II
 *   - 1D planar RF capacitive discharge, absorbing electrodes,
 *     MCC of electrons and ions with the neutral gas ............ Sec. III
 * What the paper leaves to earlier work (the explicit leap-frog cycle, the
 * direct-implicit D1 push, the MCC) is written here from the standard
 * published forms named at each function; the readings taken are listed in
 * the design notes of the repository.
 *
 * Order m: linear S_1 charge weighting and own-cell S_0 field interpolation
 * (m = 2 counted as spline order).  The MC scheme uses S_1 for both, with the
 * nodal field averaged from the two neighbouring half-grid values.
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define QE_C 1.602176634e-19     /* elementary charge, C (CODATA 2018)  */
#define EPS0 8.8541878128e-12    /* vacuum permittivity, F/m            */
#define KB_J 1.380649e-23        /* Boltzmann constant, J/K             */
#define TWO_PI 6.283185307179586476925286766559

#define MAX_PROC 8

typedef struct {
    int32_t sp, kind, n;
    double thr, e0, de;
    double* sigma;
} proc_t;

typedef struct {
    double q, m, w;
    int64_t n, cap;
    double *xi, *vx, *vy, *vz, *abar;
    uint64_t* id;
    int64_t* wait;       /* null-collision waiting time (see orc_mcc_wait_step) */
    int32_t wait_given;  /* waits supplied by the caller (else drawn by prepare) */
} species_t;

struct orc_sim {
    orc_case c;
    double dx;
    int64_t step;
    species_t sp[2];
    int32_t n_proc;
    proc_t proc[MAX_PROC];
    double numax[2];
    double pnull[2];
    double inv_log1mp[2];  /* 1 / ln(1 - P_null) */
    /* fields of the most recent solve */
    double *rho, *phi, *E, *chi, *Q[2], *cnt[2];
    double* chw[2];        /* m = 2 implicit: the operator's diagonal (uniform grid) or its
                              row sums (nonuniform grid) per centre */
    double* cho[2];        /* m = 2 implicit: the operator's coupling of centres j, j+1 */
    double *xd, *xo;       /* m = 2 implicit: the scaled operator (sum over species) */
    double *cw, *edge;     /* nonuniform grid: cell widths, node positions (m)  */
    double* sigma;         /* nonuniform grid: node charge per area (C/m^2)     */
    double* heat[2];
    const double* ext_E;   /* when set, the next step uses this field (N values) */
    orc_ledger led;
};

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11.  Ten rounds of the Philox S-box on a 128-bit    */
/* counter with a 64-bit key bumped by the Weyl constants between rounds.   */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double orc_u01(uint32_t r)
{
    return (2.0 * (double)(r >> 9) + 1.0) * (1.0 / 16777216.0);
}

/* draw d of species sp for particle id at step: ctr = (id_lo, id_hi, step, sp<<28 | d) */
static void draw4(const orc_sim* s, int32_t sp, uint64_t id, int64_t step, uint32_t d,
                  double u[4])
{
    uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), (uint32_t)step,
                       ((uint32_t)sp << 28) | d};
    uint32_t key[2] = {(uint32_t)s->c.seed, (uint32_t)(s->c.seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    for (int k = 0; k < 4; ++k) u[k] = orc_u01(r[k]);
}

static uint64_t child_id(const orc_sim* s, uint64_t parent, int64_t step, int32_t sp_child)
{
    uint32_t ctr[4] = {(uint32_t)parent, (uint32_t)(parent >> 32), (uint32_t)step,
                       ((uint32_t)sp_child << 28) | 0x0FFFFFFu};
    uint32_t key[2] = {(uint32_t)s->c.seed, (uint32_t)(s->c.seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    return ((uint64_t)r[0] | ((uint64_t)r[1] << 32)) | (1ull << 63);
}

/* ------------------------------------------------------------------------ */
/* Eq. (2) with S_1: a particle at xi in cell j = floor(xi), f = xi - j,    */
/* gives 1-f to node j and f to node j+1 (S_1(x) = 1-|x| for |x| < 1).     */
/* ------------------------------------------------------------------------ */
void orc_deposit_linear(int32_t N, int32_t periodic, int64_t n, const double* xi, double* Q)
{
    for (int64_t p = 0; p < n; ++p) {
        double j = floor(xi[p]);
        double f = xi[p] - j;
        int64_t jj = (int64_t)j;
        Q[jj] += 1.0 - f;
        Q[jj + 1] += f;
    }
    if (periodic) {
        Q[0] += Q[N];
        Q[N] = Q[0];
    }
}

void orc_count_cells(int32_t N, int64_t n, const double* xi, double* cnt)
{
    (void)N;
    for (int64_t p = 0; p < n; ++p) cnt[(int64_t)floor(xi[p])] += 1.0;
}

/* ------------------------------------------------------------------------ */
/* Dirichlet field solve by Gaussian elimination of the tridiagonal system  */
/* (Thomas algorithm).  For g = 1..N-1:                                     */
/*   -(eps0/dx^2) [ (1+chi_g)(phi_{g+1}-phi_g) - (1+chi_{g-1})(phi_g-phi_{g-1}) ] = rho_g */
/* with phi_0, phi_N given; chi = 0 is the ordinary Poisson equation of the */
/* explicit cycle, chi != 0 the susceptibility-modified operator of the     */
/* direct-implicit cycle.  E_{j+1/2} = (phi_j - phi_{j+1}) / dx.             */
/* ------------------------------------------------------------------------ */
void orc_solve_dirichlet(int32_t N, double dx, const double* rho, const double* chi,
                         double phi0, double phiN, double* phi, double* E)
{
    phi[0] = phi0;
    phi[N] = phiN;
    int32_t m = N - 1; /* unknowns phi_1..phi_{N-1} */
    if (m > 0) {
        double* a = (double*)malloc(sizeof(double) * (size_t)m);
        double* b = (double*)malloc(sizeof(double) * (size_t)m);
        double* c = (double*)malloc(sizeof(double) * (size_t)m);
        double* d = (double*)malloc(sizeof(double) * (size_t)m);
        for (int32_t g = 1; g <= m; ++g) {
            double kl = 1.0 + (chi ? chi[g - 1] : 0.0); /* (1+chi) of cell g-1 */
            double kr = 1.0 + (chi ? chi[g] : 0.0);     /* (1+chi) of cell g   */
            a[g - 1] = -kl;
            b[g - 1] = kl + kr;
            c[g - 1] = -kr;
            d[g - 1] = rho[g] * dx * dx / EPS0;
        }
        d[0] -= a[0] * phi0;
        d[m - 1] -= c[m - 1] * phiN;
        /* forward elimination */
        for (int32_t i = 1; i < m; ++i) {
            double w = a[i] / b[i - 1];
            b[i] -= w * c[i - 1];
            d[i] -= w * d[i - 1];
        }
        /* back substitution */
        phi[m] = d[m - 1] / b[m - 1];
        for (int32_t i = m - 2; i >= 0; --i) phi[i + 1] = (d[i] - c[i] * phi[i + 2]) / b[i];
        free(a); free(b); free(c); free(d);
    }
    for (int32_t j = 0; j < N; ++j) E[j] = (phi[j] - phi[j + 1]) / dx;
}

void orc_solve_dirichlet_nu(int32_t N, const double* w, const double* sigma, const double* chi,
                            double phi0, double phiN, double* phi, double* E)
{
    phi[0] = phi0;
    phi[N] = phiN;
    int32_t m = N - 1;
    if (m > 0) {
        double* a = (double*)malloc(sizeof(double) * (size_t)m);
        double* b = (double*)malloc(sizeof(double) * (size_t)m);
        double* c = (double*)malloc(sizeof(double) * (size_t)m);
        double* d = (double*)malloc(sizeof(double) * (size_t)m);
        for (int32_t g = 1; g <= m; ++g) {
            double kl = (1.0 + (chi ? chi[g - 1] : 0.0)) / w[g - 1];
            double kr = (1.0 + (chi ? chi[g] : 0.0)) / w[g];
            a[g - 1] = -kl;
            b[g - 1] = kl + kr;
            c[g - 1] = -kr;
            d[g - 1] = sigma[g] / EPS0;
        }
        d[0] -= a[0] * phi0;
        d[m - 1] -= c[m - 1] * phiN;
        for (int32_t i = 1; i < m; ++i) {
            double f = a[i] / b[i - 1];
            b[i] -= f * c[i - 1];
            d[i] -= f * d[i - 1];
        }
        phi[m] = d[m - 1] / b[m - 1];
        for (int32_t i = m - 2; i >= 0; --i) phi[i + 1] = (d[i] - c[i] * phi[i + 2]) / b[i];
        free(a); free(b); free(c); free(d);
    }
    for (int32_t j = 0; j < N; ++j) E[j] = (phi[j] - phi[j + 1]) / w[j];
}

/* ------------------------------------------------------------------------ */
/* Periodic field solve.  Gauss's law between neighbouring half-grid points */
/*   D_{j+1/2} - D_{j-1/2} = dx rho_j,  D = eps0 (1+chi) E,                  */
/* fixes D up to one constant; a periodic potential needs sum_j E dx = 0,   */
/* which fixes it.  The potential is set to zero at node 0.                 */
/* ------------------------------------------------------------------------ */
void orc_solve_periodic(int32_t N, double dx, const double* rho, const double* chi,
                        double* phi, double* E)
{
    double* P = (double*)malloc(sizeof(double) * (size_t)N);
    P[0] = 0.0;
    for (int32_t j = 1; j < N; ++j) P[j] = P[j - 1] + dx * rho[j];
    double num = 0.0, den = 0.0;
    for (int32_t j = 0; j < N; ++j) {
        double k = EPS0 * (1.0 + (chi ? chi[j] : 0.0));
        num += P[j] / k;
        den += 1.0 / k;
    }
    double D0 = -num / den;
    for (int32_t j = 0; j < N; ++j) E[j] = (D0 + P[j]) / (EPS0 * (1.0 + (chi ? chi[j] : 0.0)));
    phi[0] = 0.0;
    for (int32_t j = 0; j < N; ++j) phi[j + 1] = phi[j] - dx * E[j];
    free(P);
}

/* Eq. (3) with S_0 on the half-grid: the field of the particle's own cell. */
double orc_gather_ec(int32_t N, const double* E, double xi)
{
    (void)N;
    return E[(int64_t)floor(xi)];
}

/* Momentum-conserving gather: nodal E_g = (E_{g-1/2} + E_{g+1/2})/2, then S_1.
 * Dirichlet end nodes take the one-sided value of their only cell. */
static double nodal_E(int32_t N, int32_t periodic, const double* E, int64_t g)
{
    if (periodic) {
        int64_t gl = (g - 1 + N) % N, gr = g % N;
        return 0.5 * (E[gl] + E[gr]);
    }
    if (g == 0) return E[0];
    if (g == N) return E[N - 1];
    return 0.5 * (E[g - 1] + E[g]);
}

double orc_gather_mc(int32_t N, int32_t periodic, const double* E, double xi)
{
    double j = floor(xi);
    double f = xi - j;
    int64_t jj = (int64_t)j;
    return (1.0 - f) * nodal_E(N, periodic, E, jj) + f * nodal_E(N, periodic, E, jj + 1);
}

/* MC gather on a nonuniform grid of cell widths w (electrodes): the nodal
 * field is the centred difference of the potential over the node's two
 * cells, (phi_{g-1} - phi_{g+1}) / (w_{g-1} + w_g), i.e. the width-weighted
 * mean of the two half-grid fields; an electrode node takes its only cell's
 * field.  Linear interpolation in the logical coordinate. */
static double nodal_E_nu(int32_t N, const double* w, const double* E, int64_t g)
{
    if (g == 0) return E[0];
    if (g == N) return E[N - 1];
    return (w[g - 1] * E[g - 1] + w[g] * E[g]) / (w[g - 1] + w[g]);
}

double orc_gather_mc_nu(int32_t N, const double* w, const double* E, double xi)
{
    double j = floor(xi);
    double f = xi - j;
    int64_t jj = (int64_t)j;
    return (1.0 - f) * nodal_E_nu(N, w, E, jj) + f * nodal_E_nu(N, w, E, jj + 1);
}

/* Eq. (2) with S_2, the quadratic B-spline: S_2(x) = 3/4 - x^2 for |x| <=
 * 1/2, (3/2 - |x|)^2 / 2 for 1/2 <= |x| <= 3/2.  The nearest node i takes
 * 3/4 - d^2, its neighbours (1/2 -+ d)^2 / 2, d = xi - i in [-1/2, 1/2). */
void orc_deposit_quadratic(int32_t N, int32_t periodic, int64_t n, const double* xi, double* Q)
{
    for (int64_t p = 0; p < n; ++p) {
        double c = floor(xi[p] + 0.5);
        double d = xi[p] - c;
        int64_t i = (int64_t)c;
        double w[3] = {0.5 * (0.5 - d) * (0.5 - d), 0.75 - d * d, 0.5 * (0.5 + d) * (0.5 + d)};
        for (int k = 0; k < 3; ++k) {
            int64_t g = i - 1 + k;
            if (periodic) {
                g = ((g % N) + N) % N;          /* node N is node 0 */
            } else {
                if (g < 0) g = 0;               /* folded into the electrode */
                if (g > N) g = N;
            }
            Q[g] += w[k];
        }
    }
    if (periodic) Q[N] = Q[0];
}

/* Eq. (3) with m = 2: sum_j E_{j+1/2} S_1(xi - (j + 1/2)). */
static double half_E(int32_t N, int32_t periodic, const double* E, int64_t j)
{
    if (periodic) return E[((j % N) + N) % N];
    if (j < 0 || j >= N) return 0.0;
    return E[j];
}

double orc_gather_ec2(int32_t N, int32_t periodic, const double* E, double xi)
{
    double k = floor(xi - 0.5);
    double t = xi - 0.5 - k;
    int64_t kk = (int64_t)k;
    return (1.0 - t) * half_E(N, periodic, E, kk) + t * half_E(N, periodic, E, kk + 1);
}

void orc_chi_weights_ec2(int32_t N, int32_t periodic, int64_t n, const double* xi, double* w)
{
    memset(w, 0, sizeof(double) * (size_t)N);
    for (int64_t p = 0; p < n; ++p) {
        /* the centres on either side: a = floor(xi - 1/2) and a + 1 */
        double k = floor(xi[p] - 0.5);
        double t = xi[p] - 0.5 - k;
        int64_t c[2] = {(int64_t)k, (int64_t)k + 1};
        double s1[2] = {1.0 - t, t};
        int in[2];
        double row = 0.0;
        for (int e = 0; e < 2; ++e) {
            if (periodic) c[e] = ((c[e] % N) + N) % N;
            in[e] = periodic || (c[e] >= 0 && c[e] < N);
            if (in[e]) row += s1[e];
        }
        for (int e = 0; e < 2; ++e)
            if (in[e]) w[c[e]] += s1[e] * row;
    }
}

/* The tridiagonal operator of the m = 2 direct-implicit scheme (see the
 * header): the S_1 weights of each particle on its two centres, multiplied
 * pairwise. */
void orc_chi_operator_ec2(int32_t N, int32_t periodic, int64_t n, const double* xi,
                          double* diag, double* off)
{
    memset(diag, 0, sizeof(double) * (size_t)N);
    memset(off, 0, sizeof(double) * (size_t)N);
    for (int64_t p = 0; p < n; ++p) {
        double k = floor(xi[p] - 0.5);
        double t = xi[p] - 0.5 - k;
        int64_t a = (int64_t)k, b = a + 1;
        double wa = 1.0 - t, wb = t;
        if (periodic) {
            a = ((a % N) + N) % N;
            b = ((b % N) + N) % N;
        }
        int ina = periodic || (a >= 0 && a < N);
        int inb = periodic || (b >= 0 && b < N);
        if (ina) diag[a] += wa * wa;
        if (inb) diag[b] += wb * wb;
        if (ina && inb) off[a] += wa * wb;
    }
}

/* Solve (D + X) y = r for two right-hand sides r0, r1, with the diagonal D
 * = dg (1 where dg is NULL) and the tridiagonal X as in
 * orc_solve_chi_tridiag.  Dirichlet: the Thomas algorithm; periodic:
 * Gaussian elimination with partial pivoting of the dense matrix. */
static void solve_one_plus_x(int32_t N, int32_t periodic, const double* dg, const double* xd,
                             const double* xo, const double* r0, const double* r1, double* y0,
                             double* y1)
{
    if (!periodic) {
        double* cp = (double*)malloc(sizeof(double) * (size_t)N);
        double* d0 = (double*)malloc(sizeof(double) * (size_t)N);
        double* d1 = (double*)malloc(sizeof(double) * (size_t)N);
        for (int32_t j = 0; j < N; ++j) {
            double a = j > 0 ? xo[j - 1] : 0.0;          /* below the diagonal */
            double b = (dg ? dg[j] : 1.0) + xd[j];
            double c = j < N - 1 ? xo[j] : 0.0;          /* above the diagonal */
            double den = j > 0 ? b - a * cp[j - 1] : b;
            cp[j] = c / den;
            d0[j] = (r0[j] - (j > 0 ? a * d0[j - 1] : 0.0)) / den;
            d1[j] = (r1[j] - (j > 0 ? a * d1[j - 1] : 0.0)) / den;
        }
        y0[N - 1] = d0[N - 1];
        y1[N - 1] = d1[N - 1];
        for (int32_t j = N - 2; j >= 0; --j) {
            y0[j] = d0[j] - cp[j] * y0[j + 1];
            y1[j] = d1[j] - cp[j] * y1[j + 1];
        }
        free(cp); free(d0); free(d1);
        return;
    }
    const size_t n = (size_t)N, w = n + 2;   /* rows of [A | r0 r1] */
    double* A = (double*)calloc(n * w, sizeof(double));
    for (int32_t j = 0; j < N; ++j) {
        int32_t k = j + 1 == N ? 0 : j + 1;
        A[(size_t)j * w + j] += (dg ? dg[j] : 1.0) + xd[j];
        A[(size_t)j * w + k] += xo[j];
        A[(size_t)k * w + j] += xo[j];
        A[(size_t)j * w + n] = r0[j];
        A[(size_t)j * w + n + 1] = r1[j];
    }
    for (size_t c = 0; c < n; ++c) {
        size_t piv = c;
        for (size_t r = c + 1; r < n; ++r)
            if (fabs(A[r * w + c]) > fabs(A[piv * w + c])) piv = r;
        if (piv != c)
            for (size_t q = 0; q < w; ++q) {
                double tmp = A[c * w + q];
                A[c * w + q] = A[piv * w + q];
                A[piv * w + q] = tmp;
            }
        for (size_t r = c + 1; r < n; ++r) {
            double f = A[r * w + c] / A[c * w + c];
            if (f == 0.0) continue;
            for (size_t q = c; q < w; ++q) A[r * w + q] -= f * A[c * w + q];
        }
    }
    for (size_t c = n; c-- > 0;) {
        double s0 = A[c * w + n], s1 = A[c * w + n + 1];
        for (size_t q = c + 1; q < n; ++q) {
            s0 -= A[c * w + q] * y0[q];
            s1 -= A[c * w + q] * y1[q];
        }
        y0[c] = s0 / A[c * w + c];
        y1[c] = s1 / A[c * w + c];
    }
    free(A);
}

void orc_solve_chi_tridiag(int32_t N, int32_t periodic, double dx, const double* rho,
                           const double* xd, const double* xo, double phi0, double* phi,
                           double* E)
{
    /* eps0 (1 + X) E = D0 + R: E = (D0 / eps0) u + v with (1 + X) u = 1 and
     * (1 + X) v = R / eps0 */
    double* one = (double*)calloc((size_t)N, sizeof(double));
    double* Re = (double*)calloc((size_t)N, sizeof(double));
    double* u = (double*)malloc(sizeof(double) * (size_t)N);
    double* v = (double*)malloc(sizeof(double) * (size_t)N);
    double R = 0.0;
    for (int32_t j = 0; j < N; ++j) {
        if (j > 0) R += dx * rho[j];
        one[j] = 1.0;
        Re[j] = R / EPS0;
    }
    solve_one_plus_x(N, periodic, NULL, xd, xo, one, Re, u, v);
    double su = 0.0, sv = 0.0;
    for (int32_t j = 0; j < N; ++j) {
        su += u[j];
        sv += v[j];
    }
    if (periodic) phi0 = 0.0;
    double D0e = (phi0 / dx - sv) / su;   /* D0 / eps0 */
    phi[0] = phi0;
    for (int32_t j = 0; j < N; ++j) {
        E[j] = D0e * u[j] + v[j];
        phi[j + 1] = phi[j] - dx * E[j];
    }
    free(one); free(Re); free(u); free(v);
}

/* The m = 2 operator on a nonuniform grid (widths w, reference dx = L/N,
 * r = w / dx): each particle's products of S_1 weights divided by r_c^2 of
 * its cell c (orc_chi_operator_ec2 on the logical coordinate). */
void orc_chi_operator_ec2_nu(int32_t N, const double* w, double dx, int64_t n,
                             const double* xi, double* diag, double* off)
{
    memset(diag, 0, sizeof(double) * (size_t)N);
    memset(off, 0, sizeof(double) * (size_t)N);
    for (int64_t p = 0; p < n; ++p) {
        double k = floor(xi[p] - 0.5);
        double t = xi[p] - 0.5 - k;
        int64_t a = (int64_t)k, b = a + 1;
        int64_t c = (int64_t)floor(xi[p]);
        if (c < 0) c = 0;
        if (c > N - 1) c = N - 1;
        double rc = w[c] / dx;
        double f = 1.0 / (rc * rc);
        double wa = 1.0 - t, wb = t;
        int ina = a >= 0 && a < N, inb = b >= 0 && b < N;
        if (ina) diag[a] += f * wa * wa;
        if (inb) diag[b] += f * wb * wb;
        if (ina && inb) off[a] += f * wa * wb;
    }
}

void orc_solve_chi_tridiag_nu(int32_t N, const double* w, double dx, const double* sigma,
                              const double* xd, const double* xo, double phi0, double* phi,
                              double* E)
{
    /* (1/r + X) F = (D0 + R) / eps0, F_j = r_j E_j: F = (D0 / eps0) u + v */
    double* dg = (double*)calloc((size_t)N, sizeof(double));
    double* one = (double*)calloc((size_t)N, sizeof(double));
    double* Re = (double*)calloc((size_t)N, sizeof(double));
    double* u = (double*)malloc(sizeof(double) * (size_t)N);
    double* v = (double*)malloc(sizeof(double) * (size_t)N);
    double R = 0.0;
    for (int32_t j = 0; j < N; ++j) {
        if (j > 0) R += sigma[j];
        dg[j] = dx / w[j];
        one[j] = 1.0;
        Re[j] = R / EPS0;
    }
    solve_one_plus_x(N, 0, dg, xd, xo, one, Re, u, v);
    double su = 0.0, sv = 0.0;
    for (int32_t j = 0; j < N; ++j) {
        su += u[j];
        sv += v[j];
    }
    double D0e = (phi0 / dx - sv) / su;   /* from dx sum_j F_j = phi_0 - phi_N */
    phi[0] = phi0;
    for (int32_t j = 0; j < N; ++j) {
        double F = D0e * u[j] + v[j];
        E[j] = F * dx / w[j];
        phi[j + 1] = phi[j] - dx * F;
    }
    free(dg); free(one); free(Re); free(u); free(v);
}

static double gather(const orc_sim* s, double xi);

/* Eq. (3) with m = 2 on a nonuniform grid (electrodes): minus the derivative
 * of the deposit's field energy with respect to the physical position,
 * (1 / w_c) sum_h (phi_h - phi_{h+1}) S_1(xi - (h + 1/2)) with c the
 * particle's cell, phi_h - phi_{h+1} = E_{h+1/2} w_h (zero beyond an
 * electrode). */
double orc_gather_ec2_nu(int32_t N, const double* w, const double* E, double xi)
{
    double k = floor(xi - 0.5);
    double t = xi - 0.5 - k;
    int64_t a = (int64_t)k, b = a + 1;
    double da = (a >= 0 && a < N) ? E[a] * w[a] : 0.0;
    double db = (b >= 0 && b < N) ? E[b] * w[b] : 0.0;
    int64_t c = (int64_t)floor(xi);
    if (c > N - 1) c = N - 1;
    return ((1.0 - t) * da + t * db) / w[c];
}

/* Ion subcycling: the time step of species sp in units of dt, and whether
 * the species moves in the current step. */
static double substep(const orc_sim* s, int sp)
{
    return (sp == 1 && s->c.ion_subcycle > 1) ? (double)s->c.ion_subcycle : 1.0;
}

static int moves(const orc_sim* s, int sp)
{
    return !(sp == 1 && s->c.ion_subcycle > 1) || s->step % s->c.ion_subcycle == 0;
}

/* The weight of species sp in the D1 susceptibility, q^2 w / m (h dt)^2 / dt^2
 * with h its time step in units of dt: a subcycled species responds only to
 * the field of the steps in which it moves (zero otherwise). */
static double chi_weight(const orc_sim* s, int sp)
{
    const species_t* p = &s->sp[sp];
    if (!(p->m > 0.0) || !moves(s, sp)) return 0.0;
    double h = substep(s, sp);
    return p->q * p->q * p->w / p->m * h * h;
}

/* ------------------------------------------------------------------------ */
/* Simulation object                                                        */
/* ------------------------------------------------------------------------ */
static void* xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

orc_sim* orc_create(const orc_case* c)
{
    if (c->n_cells < 2) return NULL;
    if (c->gather < ORC_GATHER_EC || c->gather > ORC_GATHER_EC2) return NULL;
    if (c->ion_subcycle < 0) return NULL;
    if (c->cell_dx_m) {
        /* nonuniform grids: between electrodes, widths summing to L */
        if (c->bc != ORC_BC_DIRICHLET) return NULL;
        double L = 0.0;
        for (int32_t j = 0; j < c->n_cells; ++j) {
            if (!(c->cell_dx_m[j] > 0.0) || !isfinite(c->cell_dx_m[j])) return NULL;
            L += c->cell_dx_m[j];
        }
        if (!(fabs(L - c->gap_m) <= 1e-9 * c->gap_m)) return NULL;
    }
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->c = *c;
    s->dx = c->gap_m / c->n_cells;
    s->c.cell_dx_m = NULL;   /* the caller's array is copied below */
    s->step = c->step0;
    int32_t N = c->n_cells;
    s->rho = (double*)xcalloc((size_t)N + 1, sizeof(double));
    s->phi = (double*)xcalloc((size_t)N + 1, sizeof(double));
    s->E = (double*)xcalloc((size_t)N, sizeof(double));
    s->chi = (double*)xcalloc((size_t)N, sizeof(double));
    s->xd = (double*)xcalloc((size_t)N, sizeof(double));
    s->xo = (double*)xcalloc((size_t)N, sizeof(double));
    for (int k = 0; k < 2; ++k) {
        s->Q[k] = (double*)xcalloc((size_t)N + 1, sizeof(double));
        s->cnt[k] = (double*)xcalloc((size_t)N, sizeof(double));
        s->chw[k] = (double*)xcalloc((size_t)N, sizeof(double));
        s->cho[k] = (double*)xcalloc((size_t)N, sizeof(double));
        s->heat[k] = (double*)xcalloc((size_t)N, sizeof(double));
    }
    if (c->cell_dx_m) {
        s->cw = (double*)xcalloc((size_t)N, sizeof(double));
        s->edge = (double*)xcalloc((size_t)N + 1, sizeof(double));
        s->sigma = (double*)xcalloc((size_t)N + 1, sizeof(double));
        for (int32_t j = 0; j < N; ++j) {
            s->cw[j] = c->cell_dx_m[j];
            s->edge[j + 1] = s->edge[j] + s->cw[j];
        }
    }
    return s;
}

void orc_destroy(orc_sim* s)
{
    if (!s) return;
    for (int k = 0; k < 2; ++k) {
        species_t* p = &s->sp[k];
        free(p->xi); free(p->vx); free(p->vy); free(p->vz); free(p->abar); free(p->id);
        free(p->wait);
        free(s->Q[k]); free(s->cnt[k]); free(s->chw[k]); free(s->cho[k]); free(s->heat[k]);
    }
    for (int k = 0; k < s->n_proc; ++k) free(s->proc[k].sigma);
    free(s->rho); free(s->phi); free(s->E); free(s->chi); free(s->xd); free(s->xo);
    free(s->cw); free(s->edge); free(s->sigma);
    free(s);
}

static void species_reserve(species_t* p, int64_t need)
{
    if (need <= p->cap) return;
    int64_t cap = p->cap ? p->cap : 16;
    while (cap < need) cap *= 2;
    p->xi = (double*)realloc(p->xi, sizeof(double) * (size_t)cap);
    p->vx = (double*)realloc(p->vx, sizeof(double) * (size_t)cap);
    p->vy = (double*)realloc(p->vy, sizeof(double) * (size_t)cap);
    p->vz = (double*)realloc(p->vz, sizeof(double) * (size_t)cap);
    p->abar = (double*)realloc(p->abar, sizeof(double) * (size_t)cap);
    p->id = (uint64_t*)realloc(p->id, sizeof(uint64_t) * (size_t)cap);
    p->wait = (int64_t*)realloc(p->wait, sizeof(int64_t) * (size_t)cap);
    p->cap = cap;
}

int orc_set_species(orc_sim* s, int32_t k, double q, double m, double w, int64_t n,
                    const double* xi, const double* vx, const double* vy, const double* vz,
                    const double* abar, const uint64_t* id, const int64_t* wait)
{
    if (k < 0 || k > 1 || n < 0 || m <= 0.0) return -1;
    species_t* p = &s->sp[k];
    p->q = q; p->m = m; p->w = w;
    species_reserve(p, n);
    p->n = n;
    for (int64_t i = 0; i < n; ++i) {
        p->xi[i] = xi[i];
        p->vx[i] = vx[i];
        p->vy[i] = vy[i];
        p->vz[i] = vz[i];
        p->abar[i] = abar ? abar[i] : 0.0;
        p->id[i] = id[i];
        p->wait[i] = wait ? wait[i] : 0;
    }
    p->wait_given = wait != NULL;
    return 0;
}

int orc_add_process(orc_sim* s, int32_t sp, int32_t kind, double thr, double e0, double de,
                    int32_t n, const double* sigma)
{
    if (s->n_proc >= MAX_PROC || n < 2 || de <= 0.0 || sp < 0 || sp > 1) return -1;
    proc_t* pr = &s->proc[s->n_proc++];
    pr->sp = sp; pr->kind = kind; pr->thr = thr; pr->e0 = e0; pr->de = de; pr->n = n;
    pr->sigma = (double*)malloc(sizeof(double) * (size_t)n);
    memcpy(pr->sigma, sigma, sizeof(double) * (size_t)n);
    return 0;
}

/* Linear interpolation of a table on e0 + k de, held constant outside it. */
static double sigma_at(const proc_t* pr, double eps)
{
    if (pr->thr > 0.0 && eps <= pr->thr) return 0.0;
    double t = (eps - pr->e0) / pr->de;
    if (t <= 0.0) return pr->sigma[0];
    if (t >= (double)(pr->n - 1)) return pr->sigma[pr->n - 1];
    int64_t k = (int64_t)floor(t);
    double f = t - (double)k;
    return (1.0 - f) * pr->sigma[k] + f * pr->sigma[k + 1];
}

/* A candidate whose energy lies past the last table point (sigma held there). */
static int beyond_table(const orc_sim* s, int32_t sp, double eps)
{
    for (int k = 0; k < s->n_proc; ++k)
        if (s->proc[k].sp == sp)
            return eps > s->proc[k].e0 + (double)(s->proc[k].n - 1) * s->proc[k].de;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Null-collision candidacy (Vahedi & Surendra 1995): in every step every   */
/* particle is a candidate independently with probability P_null.  The      */
/* Bernoulli sequence is realised by geometric waiting times: a particle    */
/* carries the number of non-candidate steps left before its next           */
/* candidacy, W ~ Geo0(P_null), P(W = k) = (1 - P_null)^k P_null, drawn by  */
/* inversion W = floor(ln u / ln(1 - P_null)) from a uniform u of the       */
/* particle's Philox stream.  W is held as a plain integer (a wait longer   */
/* than 2^63 steps, possible only for P_null below about 2e-18, is held as  */
/* the largest int64: never reached).                                       */
/* ------------------------------------------------------------------------ */
static int64_t geo0(const orc_sim* s, int32_t sp, double u)
{
    if (s->pnull[sp] >= 1.0) return 0;
    double W = floor(log(u) * s->inv_log1mp[sp]);
    return W < 9.0e18 ? (int64_t)W : INT64_MAX;
}

int64_t orc_mcc_first_wait(const orc_sim* s, int32_t sp, uint64_t id, int64_t step)
{
    double u[4];
    draw4(s, sp, id, step, 4, u);
    return geo0(s, sp, u[0]);
}

int orc_mcc_wait_step(const orc_sim* s, int32_t sp, uint64_t id, int64_t step, int64_t* wait)
{
    if (*wait > 0) {
        *wait -= 1;
        return 0;
    }
    /* candidate: the next waiting time comes from u0 of draw 0 */
    double u[4];
    draw4(s, sp, id, step, 0, u);
    *wait = geo0(s, sp, u[0]);
    return 1;
}

/* Null-collision frequency (Vahedi & Surendra, Comput. Phys. Commun. 87 (1995)
 * 179): an upper bound of n_g sigma_T(eps) |v(eps)| over the tabulated range,
 * taken interval by interval.  For ions |v| is the relative speed g with
 * eps = M g^2 / 2. */
int orc_prepare(orc_sim* s)
{
    for (int sp = 0; sp < 2; ++sp) {
        s->numax[sp] = 0.0;
        int first = -1;
        for (int k = 0; k < s->n_proc; ++k) {
            if (s->proc[k].sp != sp) continue;
            if (first < 0) first = k;
            const proc_t* a = &s->proc[first];
            const proc_t* b = &s->proc[k];
            if (a->n != b->n || a->e0 != b->e0 || a->de != b->de) return -1;
            if (sp == 1 && b->kind != ORC_CHARGE_EXCHANGE) return -1;
            if (sp == 0 && b->kind == ORC_CHARGE_EXCHANGE) return -1;
        }
        if (first < 0) { s->pnull[sp] = 0.0; continue; }
        const proc_t* a = &s->proc[first];
        double mass = s->sp[sp].m;
        double best = 0.0;
        for (int32_t i = 0; i + 1 < a->n; ++i) {
            double sl = 0.0, sr = 0.0;
            for (int k = 0; k < s->n_proc; ++k) {
                if (s->proc[k].sp != sp) continue;
                sl += s->proc[k].sigma[i];
                sr += s->proc[k].sigma[i + 1];
            }
            double er = a->e0 + (double)(i + 1) * a->de;
            double v = sqrt(2.0 * QE_C * (er > 0.0 ? er : 0.0) / mass);
            double cand = (sl > sr ? sl : sr) * v;
            if (cand > best) best = cand;
        }
        s->numax[sp] = s->c.gas_density_m3 * best;
        s->pnull[sp] = 1.0 - exp(-s->numax[sp] * s->c.dt_s * substep(s, sp));
    }
    for (int sp = 0; sp < 2; ++sp) {
        double p = s->pnull[sp];
        s->inv_log1mp[sp] = (p > 0.0 && p < 1.0) ? 1.0 / log1p(-p) : 0.0;
        /* particles loaded without waits take their first trial at step0 */
        species_t* q = &s->sp[sp];
        if (!q->wait_given)
            for (int64_t i = 0; i < q->n; ++i) q->wait[i] = orc_mcc_first_wait(s, sp, q->id[i], s->step);
    }
    return 0;
}

double orc_numax(const orc_sim* s, int32_t sp) { return s->numax[sp]; }

static double rf_volts_at(const orc_sim* s, int64_t step)
{
    double t = (double)step * s->c.dt_s;
    return s->c.rf_volts * sin(TWO_PI * s->c.rf_freq_hz * t);
}

/* Deposit both species at their stored positions and solve.  phi_0 is
 * V(t_{step_for_bc}); chi is used for the implicit operator. */
static void fields(orc_sim* s, int use_chi, int64_t step_for_bc)
{
    int32_t N = s->c.n_cells;
    int periodic = s->c.bc == ORC_BC_PERIODIC;
    if (s->ext_E) {
        /* field supplied by the caller (a sample of a larger discharge) */
        double we = 0.0;
        for (int32_t j = 0; j < N; ++j) {
            s->E[j] = s->ext_E[j];
            we += 0.5 * EPS0 * s->E[j] * s->E[j] * (s->cw ? s->cw[j] : s->dx);
        }
        s->led.WE = we;
        return;
    }
    for (int k = 0; k < 2; ++k) {
        memset(s->Q[k], 0, sizeof(double) * ((size_t)N + 1));
        memset(s->cnt[k], 0, sizeof(double) * (size_t)N);
        if (s->c.gather == ORC_GATHER_EC2)
            orc_deposit_quadratic(N, periodic, s->sp[k].n, s->sp[k].xi, s->Q[k]);
        else
            orc_deposit_linear(N, periodic, s->sp[k].n, s->sp[k].xi, s->Q[k]);
        orc_count_cells(N, s->sp[k].n, s->sp[k].xi, s->cnt[k]);
        if (use_chi && s->c.gather == ORC_GATHER_EC2) {
            if (s->cw)
                orc_chi_operator_ec2_nu(N, s->cw, s->dx, s->sp[k].n, s->sp[k].xi, s->chw[k],
                                        s->cho[k]);
            else
                orc_chi_operator_ec2(N, periodic, s->sp[k].n, s->sp[k].xi, s->chw[k],
                                     s->cho[k]);
        }
    }
    for (int32_t g = 0; g <= N; ++g) {
        double r = s->c.background_rho;
        if (s->cw) {
            /* charge per area of node g; rho over the node's volume: half
             * of each adjacent cell, the whole end cell at an electrode */
            double vol = g == 0 ? s->cw[0]
                       : g == N ? s->cw[N - 1] : 0.5 * (s->cw[g - 1] + s->cw[g]);
            double sg = r * vol;
            for (int k = 0; k < 2; ++k) sg += s->sp[k].q * s->sp[k].w * s->Q[k][g];
            s->sigma[g] = sg;
            s->rho[g] = sg / vol;
            continue;
        }
        for (int k = 0; k < 2; ++k) r += s->sp[k].q * s->sp[k].w * s->Q[k][g] / s->dx;
        s->rho[g] = r;
    }
    /* EC: chi_{j+1/2} = beta dt^2 / (eps0 dx) * sum_s q_s^2 w_s / m_s * N_{s,j},
     * beta = 1/2, with N_{s,j} the count of predicted particles in cell j.
     * MC: the susceptibility of the linear (CIC) weights at the nodes,
     * chi_g = beta dt^2 / eps0 * sum_s q_s^2 w_s / m_s * Q_{s,g} / V_g (V_g = dx,
     * dx/2 at Dirichlet electrodes), and
     * chi_{j+1/2} = (chi_j + chi_{j+1}) / 2.
     * EC with m = 2: the tridiagonal operator beta dt^2 / (eps0 dx) * sum_s
     * q_s^2 w_s / m_s * M_s (orc_chi_operator_ec2), solved as such; chi
     * holds its row sums.  On a nonuniform grid the operator acts on
     * F_j = r_j E_j (orc_chi_operator_ec2_nu, orc_solve_chi_tridiag_nu) and
     * chi_j = sum_j' X_jj' r_j' (the susceptibility of a uniform field). */
    const int ec2_exact = use_chi && s->c.gather == ORC_GATHER_EC2;
    if (ec2_exact) {
        const double coef = 0.5 * s->c.dt_s * s->c.dt_s / (EPS0 * s->dx);
        for (int32_t j = 0; j < N; ++j) {
            double d = 0.0, o = 0.0;
            for (int k = 0; k < 2; ++k) {
                double f = chi_weight(s, k);
                d += f * s->chw[k][j];
                o += f * s->cho[k][j];
            }
            s->xd[j] = coef * d;
            s->xo[j] = coef * o;
        }
        if (s->cw) {
            for (int32_t j = 0; j < N; ++j) {
                double x = s->xd[j] * s->cw[j];
                if (j > 0) x += s->xo[j - 1] * s->cw[j - 1];
                if (j < N - 1) x += s->xo[j] * s->cw[j + 1];
                s->chi[j] = x / s->dx;
            }
            orc_solve_chi_tridiag_nu(N, s->cw, s->dx, s->sigma, s->xd, s->xo,
                                     rf_volts_at(s, step_for_bc), s->phi, s->E);
        } else {
            for (int32_t j = 0; j < N; ++j) {
                double left = j > 0 ? s->xo[j - 1] : (periodic ? s->xo[N - 1] : 0.0);
                s->chi[j] = s->xd[j] + s->xo[j] + left;
            }
            orc_solve_chi_tridiag(N, periodic, s->dx, s->rho, s->xd, s->xo,
                                  periodic ? 0.0 : rf_volts_at(s, step_for_bc), s->phi, s->E);
        }
        double we = 0.0;
        for (int32_t j = 0; j < N; ++j)
            we += 0.5 * EPS0 * s->E[j] * s->E[j] * (s->cw ? s->cw[j] : s->dx);
        s->led.WE = we;
        return;
    }
    for (int32_t j = 0; j < N; ++j) {
        double x = 0.0;
        if (use_chi && s->c.gather == ORC_GATHER_MC) {
            for (int32_t g = j; g <= j + 1; ++g) {
                double vol = s->dx;
                if (!periodic && (g == 0 || g == N)) vol = 0.5 * s->dx;
                if (s->cw)   /* half of each adjacent cell */
                    vol = 0.5 * ((g > 0 ? s->cw[g - 1] : 0.0) + (g < N ? s->cw[g] : 0.0));
                /* the periodic deposit holds the folded node in Q_0 and Q_N */
                for (int k = 0; k < 2; ++k) x += 0.5 * chi_weight(s, k) * s->Q[k][g] / vol;
            }
            s->chi[j] = 0.5 * s->c.dt_s * s->c.dt_s / EPS0 * x;
            continue;
        }
        if (use_chi)
            for (int k = 0; k < 2; ++k) x += chi_weight(s, k) * s->cnt[k][j];
        s->chi[j] = 0.5 * s->c.dt_s * s->c.dt_s / (EPS0 * (s->cw ? s->cw[j] : s->dx)) * x;
    }
    if (periodic)
        orc_solve_periodic(N, s->dx, s->rho, use_chi ? s->chi : NULL, s->phi, s->E);
    else if (s->cw)
        orc_solve_dirichlet_nu(N, s->cw, s->sigma, use_chi ? s->chi : NULL,
                               rf_volts_at(s, step_for_bc), 0.0, s->phi, s->E);
    else
        orc_solve_dirichlet(N, s->dx, s->rho, use_chi ? s->chi : NULL,
                            rf_volts_at(s, step_for_bc), 0.0, s->phi, s->E);
    double we = 0.0;
    for (int32_t j = 0; j < N; ++j)
        we += 0.5 * EPS0 * s->E[j] * s->E[j] * (s->cw ? s->cw[j] : s->dx);
    s->led.WE = we;
}

int orc_compute_fields(orc_sim* s)
{
    int imp = s->c.scheme == ORC_IMPLICIT;
    fields(s, imp, imp ? s->step + 1 : s->step);
    return 0;
}

static double kin(const species_t* p, double vx, double vy, double vz)
{
    return 0.5 * p->m * p->w * (vx * vx + vy * vy + vz * vz);
}

static void remove_particle(species_t* p, int64_t i)
{
    int64_t last = p->n - 1;
    p->xi[i] = p->xi[last]; p->vx[i] = p->vx[last]; p->vy[i] = p->vy[last];
    p->vz[i] = p->vz[last]; p->abar[i] = p->abar[last]; p->id[i] = p->id[last];
    p->wait[i] = p->wait[last];
    p->n = last;
}

static void append_particle(species_t* p, double xi, double vx, double vy, double vz,
                            double abar, uint64_t id, int64_t wait)
{
    species_reserve(p, p->n + 1);
    int64_t i = p->n++;
    p->xi[i] = xi; p->vx[i] = vx; p->vy[i] = vy; p->vz[i] = vz; p->abar[i] = abar;
    p->id[i] = id;
    p->wait[i] = wait;
}

/* A move by the physical distance d (m) on a nonuniform grid: the physical
 * position X = e_c + (xi - c) w_c is moved and mapped back to the cell whose
 * edges hold it (bisection over the node positions); beyond an electrode
 * the width of the cell next to it continues the map, so that the boundary
 * rule below absorbs the particle.  (On a uniform grid xi += d / dx.) */
static void move_nonuniform(const orc_sim* s, double* xi, double d)
{
    int32_t N = s->c.n_cells;
    int32_t c = (int32_t)floor(*xi);
    double X = s->edge[c] + (*xi - c) * s->cw[c] + d;
    if (X < 0.0) { *xi = X / s->cw[0]; return; }
    if (X >= s->edge[N]) { *xi = N + (X - s->edge[N]) / s->cw[N - 1]; return; }
    int32_t lo = 0, hi = N;   /* edge[lo] <= X < edge[hi] */
    while (hi - lo > 1) {
        int32_t mid = (lo + hi) / 2;
        if (s->edge[mid] <= X) lo = mid;
        else hi = mid;
    }
    *xi = lo + (X - s->edge[lo]) / s->cw[lo];
}

/* Boundary rule.  Dirichlet: absorbed at the electrode it crossed
 * (returns 0 for x=0, 1 for x=L), else -1.  Periodic: wrapped, returns -1. */
static int boundary(const orc_sim* s, double* xi)
{
    double N = (double)s->c.n_cells;
    if (s->c.bc == ORC_BC_PERIODIC) {
        while (*xi < 0.0) *xi += N;
        while (*xi >= N) *xi -= N;
        return -1;
    }
    if (*xi < 0.0) return 0;
    if (*xi >= N) return 1;
    return -1;
}

/* Isotropic unit vector: cos(theta) = 1 - 2 ua, azimuth 2 pi ub. */
static void iso_dir(double ua, double ub, double d[3])
{
    double ct = 1.0 - 2.0 * ua;
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double ph = TWO_PI * ub;
    d[0] = st * cos(ph);
    d[1] = st * sin(ph);
    d[2] = ct;
}

/* Box-Muller pair from (ua, ub). */
static void box_muller(double ua, double ub, double* n1, double* n2)
{
    double r = sqrt(-2.0 * log(ua));
    *n1 = r * cos(TWO_PI * ub);
    *n2 = r * sin(TWO_PI * ub);
}

/* ------------------------------------------------------------------------ */
/* Null-collision MCC of one particle (Vahedi & Surendra 1995), at most one */
/* real collision per step.  Random numbers: Philox draw 0 (candidacy u0,   */
/* process u1, scattering angles u2 u3), draw 1 (ionization energy sharing  */
/* u0, ejected-electron angles u1 u2), draw 2 (neutral velocity of the ion  */
/* collision), draw 3 (velocity of the new ion).                            */
/* ------------------------------------------------------------------------ */
int orc_collide_one(orc_sim* s, int32_t sp, uint64_t id, int64_t step, double* v,
                    double* ve, double* vi, int* eps_over)
{
    double u[4];
    draw4(s, sp, id, step, 0, u);
    const species_t* me = &s->sp[sp];
    double ng = s->c.gas_density_m3;
    double vth_gas = sqrt(KB_J * s->c.gas_temp_K / s->c.gas_mass_kg);
    if (sp == 0) {
        double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        double vm = sqrt(v2);
        double eps = 0.5 * me->m * v2 / QE_C;
        if (eps_over) *eps_over = beyond_table(s, 0, eps);
        double cum = 0.0;
        int chosen = -1;
        for (int k = 0; k < s->n_proc; ++k) {
            if (s->proc[k].sp != 0) continue;
            double sig = sigma_at(&s->proc[k], eps);
            cum += ng * sig * vm / s->numax[0];
            if (u[1] < cum) { chosen = k; break; }
        }
        if (chosen < 0) return -2;
        const proc_t* pr = &s->proc[chosen];
        double d[3];
        iso_dir(u[2], u[3], d);
        if (pr->kind == ORC_ELASTIC) {
            double cchi = vm > 0.0 ? (v[0] * d[0] + v[1] * d[1] + v[2] * d[2]) / vm : 0.0;
            double e1 = eps * (1.0 - 2.0 * me->m / s->c.gas_mass_kg * (1.0 - cchi));
            double sp1 = sqrt(2.0 * QE_C * e1 / me->m);
            for (int k = 0; k < 3; ++k) v[k] = sp1 * d[k];
        } else if (pr->kind == ORC_EXCITATION) {
            double e1 = eps - pr->thr;
            double sp1 = sqrt(2.0 * QE_C * e1 / me->m);
            for (int k = 0; k < 3; ++k) v[k] = sp1 * d[k];
        } else { /* ionization */
            double u1[4], u3[4];
            draw4(s, sp, id, step, 1, u1);
            draw4(s, sp, id, step, 3, u3);
            double B = s->c.opal_B_eV;
            double avail = eps - pr->thr;
            /* Opal, Peterson & Beaty energy sharing: eps_ej = B tan(u atan(avail/(2B))) */
            double eej = B * tan(u1[0] * atan(avail / (2.0 * B)));
            double esc = avail - eej;
            double sp1 = sqrt(2.0 * QE_C * esc / me->m);
            for (int k = 0; k < 3; ++k) v[k] = sp1 * d[k];
            double d2[3];
            iso_dir(u1[1], u1[2], d2);
            double sp2 = sqrt(2.0 * QE_C * eej / me->m);
            for (int k = 0; k < 3; ++k) ve[k] = sp2 * d2[k];
            double n1, n2, n3, n4;
            box_muller(u3[0], u3[1], &n1, &n2);
            box_muller(u3[2], u3[3], &n3, &n4);
            double vti = sqrt(KB_J * s->c.gas_temp_K / s->sp[1].m);
            vi[0] = vti * n1; vi[1] = vti * n2; vi[2] = vti * n3;
        }
        return pr->kind;
    }
    /* ions: charge exchange against a neutral drawn from the gas Maxwellian */
    double u2[4];
    draw4(s, sp, id, step, 2, u2);
    double n1, n2, n3, n4;
    box_muller(u2[0], u2[1], &n1, &n2);
    box_muller(u2[2], u2[3], &n3, &n4);
    double vn[3] = {vth_gas * n1, vth_gas * n2, vth_gas * n3};
    double gx = v[0] - vn[0], gy = v[1] - vn[1], gz = v[2] - vn[2];
    double g2 = gx * gx + gy * gy + gz * gz;
    double g = sqrt(g2);
    double eg = 0.5 * me->m * g2 / QE_C;
    if (eps_over) *eps_over = beyond_table(s, 1, eg);
    double cum = 0.0;
    for (int k = 0; k < s->n_proc; ++k) {
        if (s->proc[k].sp != 1) continue;
        double sig = sigma_at(&s->proc[k], eg);
        cum += ng * sig * g / s->numax[1];
        if (u[1] < cum) {
            v[0] = vn[0]; v[1] = vn[1]; v[2] = vn[2];
            return ORC_CHARGE_EXCHANGE;
        }
    }
    return -2;
}

/* MCC over the first n0 particles of species sp (those present before the
 * collision stage: children born in this step do not collide in it);
 * children are appended (electron to species 0, ion to species 1). */
static void mcc_species(orc_sim* s, int32_t sp, int64_t n0, int64_t step)
{
    species_t* p = &s->sp[sp];
    if (!(s->pnull[sp] > 0.0)) return;
    for (int64_t i = 0; i < n0; ++i) {
        if (!orc_mcc_wait_step(s, sp, p->id[i], step, &p->wait[i])) continue;
        s->led.n_candidates[sp]++;
        double v[3] = {p->vx[i], p->vy[i], p->vz[i]};
        double ve[3], vi[3];
        int over = 0;
        double k0 = kin(p, v[0], v[1], v[2]);
        int r = orc_collide_one(s, sp, p->id[i], step, v, ve, vi, &over);
        if (over) s->led.n_over_table[sp]++;
        if (r < 0) continue;
        s->led.n_coll[sp][r]++;
        p->vx[i] = v[0]; p->vy[i] = v[1]; p->vz[i] = v[2];
        s->led.coll_dK[sp] += kin(p, v[0], v[1], v[2]) - k0;
        if (r == ORC_IONIZATION) {
            uint64_t ide = child_id(s, p->id[i], step, 0);
            uint64_t idi = child_id(s, p->id[i], step, 1);
            double x = p->xi[i];
            append_particle(&s->sp[0], x, ve[0], ve[1], ve[2], 0.0, ide,
                            orc_mcc_first_wait(s, 0, ide, step));
            append_particle(&s->sp[1], x, vi[0], vi[1], vi[2], 0.0, idi,
                            orc_mcc_first_wait(s, 1, idi, step));
            s->led.coll_dK[0] += kin(&s->sp[0], ve[0], ve[1], ve[2]);
            s->led.coll_dK[1] += kin(&s->sp[1], vi[0], vi[1], vi[2]);
            s->led.n_created[0]++;
            s->led.n_created[1]++;
        }
    }
}

static void mcc_all(orc_sim* s)
{
    int64_t n0 = s->sp[0].n, n1 = s->sp[1].n;
    mcc_species(s, 0, n0, s->step);
    if (moves(s, 1)) mcc_species(s, 1, n1, s->step);
}

static void begin_ledger(orc_sim* s, int implicit)
{
    double we = s->led.WE;
    memset(&s->led, 0, sizeof(s->led));
    s->led.WE = we;
    for (int k = 0; k < 2; ++k) {
        species_t* p = &s->sp[k];
        double K = 0.0;
        /* implicit state stores v~ = v_{n-1/2} + h dt abar/2 */
        double hdt = s->c.dt_s * substep(s, k);
        for (int64_t i = 0; i < p->n; ++i) {
            double vx = implicit ? p->vx[i] - 0.5 * hdt * p->abar[i] : p->vx[i];
            K += kin(p, vx, p->vy[i], p->vz[i]);
        }
        s->led.K_before[k] = K;
    }
}

/* Kinetic energy at n+1/2; a species that stood in an implicit step still
 * holds its prediction, v~ = v + h dt abar/2. */
static void end_ledger(orc_sim* s, int implicit)
{
    for (int k = 0; k < 2; ++k) {
        species_t* p = &s->sp[k];
        const int held = implicit && !moves(s, k);
        double hdt = s->c.dt_s * substep(s, k);
        double K = 0.0;
        for (int64_t i = 0; i < p->n; ++i) {
            double vx = held ? p->vx[i] - 0.5 * hdt * p->abar[i] : p->vx[i];
            K += kin(p, vx, p->vy[i], p->vz[i]);
        }
        s->led.K_after[k] = K;
    }
}

/* ------------------------------------------------------------------------ */
/* Explicit cycle n -> n+1 (leap-frog): deposit xi_n (Eq. 2), solve with    */
/* phi_0 = V(t_n), gather (Eq. 3 for EC, CIC for MC), push, absorb/wrap,    */
/* MCC on v_{n+1/2}.                                                        */
/* ------------------------------------------------------------------------ */
/* the field at a particle, by the case's gather */
static double gather(const orc_sim* s, double xi)
{
    int32_t N = s->c.n_cells;
    int periodic = s->c.bc == ORC_BC_PERIODIC;
    if (s->c.gather == ORC_GATHER_MC && s->cw) return orc_gather_mc_nu(N, s->cw, s->E, xi);
    if (s->c.gather == ORC_GATHER_MC) return orc_gather_mc(N, periodic, s->E, xi);
    if (s->c.gather == ORC_GATHER_EC2 && s->cw) return orc_gather_ec2_nu(N, s->cw, s->E, xi);
    if (s->c.gather == ORC_GATHER_EC2) return orc_gather_ec2(N, periodic, s->E, xi);
    return orc_gather_ec(N, s->E, xi);
}

static void step_explicit(orc_sim* s)
{
    fields(s, 0, s->step);
    begin_ledger(s, 0);
    for (int k = 0; k < 2; ++k) {
        species_t* p = &s->sp[k];
        if (!moves(s, k)) continue;   /* a subcycled species stands */
        double h = substep(s, k);     /* the species' time step in units of dt */
        double qm_dt = p->q / p->m * s->c.dt_s * h;
        double dt_dx = s->c.dt_s / s->dx * h;
        int64_t i = 0;
        while (i < p->n) {
            double Ep = gather(s, p->xi[i]);
            double dv = qm_dt * Ep;
            /* 1/2 m (v+dv)^2 - 1/2 m v^2 written without cancellation */
            double dK = p->m * p->w * dv * (p->vx[i] + 0.5 * dv);
            s->led.work[k] += dK;
            s->heat[k][(int64_t)floor(p->xi[i])] += dK;
            p->vx[i] += dv;
            if (s->cw) move_nonuniform(s, &p->xi[i], p->vx[i] * s->c.dt_s * h);
            else p->xi[i] += p->vx[i] * dt_dx;
            int e = boundary(s, &p->xi[i]);
            if (e >= 0) {
                s->led.absorbed_n[k][e]++;
                s->led.absorbed_K[k][e] += kin(p, p->vx[i], p->vy[i], p->vz[i]);
                remove_particle(p, i);
                continue;
            }
            ++i;
        }
    }
    if (s->c.collisions) mcc_all(s);
    end_ledger(s, 0);
    s->step++;
}

/* ------------------------------------------------------------------------ */
/* Direct-implicit D1 cycle (Langdon, Cohen & Friedman, J. Comput. Phys. 51  */
/* (1983) 107; beta = 1/2).  Stored: x~_{n+1}, v~ = v_{n-1/2} + dt abar/2,  */
/* abar_{n-1}.  Deposit rho~ and the cell counts at x~, solve the           */
/* susceptibility-modified equation with phi_0 = V(t_{n+1}), then           */
/*   a = (q/m) E(x~),  x_{n+1} = x~ + beta dt^2 a,  v_{n+1/2} = v~ + beta dt a, */
/*   abar_n = (abar_{n-1} + a)/2,                                            */
/* absorb at x_{n+1}, MCC on v_{n+1/2}, and predict the next step:          */
/*   v~' = v_{n+1/2} + dt abar_n / 2,  x~_{n+2} = x_{n+1} + dt v~'           */
/* (a prediction outside the gap is absorbed at once).                      */
/* Subcycled ions take the cycle with h dt in place of dt in the steps in   */
/* which they move and stand in the others (their prediction held, their    */
/* susceptibility left out of the solve).                                   */
/* ------------------------------------------------------------------------ */
static void step_implicit(orc_sim* s)
{
    fields(s, 1, s->step + 1);
    begin_ledger(s, 1);
    for (int k = 0; k < 2; ++k) {
        species_t* p = &s->sp[k];
        if (!moves(s, k)) continue;
        double dt = s->c.dt_s * substep(s, k);
        double qm = p->q / p->m;
        int64_t i = 0;
        while (i < p->n) {
            double Ep = gather(s, p->xi[i]);
            double a = qm * Ep;
            double vold = p->vx[i] - 0.5 * dt * p->abar[i];    /* v_{n-1/2}  */
            double vnew = p->vx[i] + 0.5 * dt * a;             /* v_{n+1/2}  */
            double dv = vnew - vold;
            double dK = p->m * p->w * dv * (vold + 0.5 * dv);
            s->led.work[k] += dK;
            s->heat[k][(int64_t)floor(p->xi[i])] += dK;
            if (s->cw) move_nonuniform(s, &p->xi[i], 0.5 * dt * dt * a);
            else p->xi[i] += 0.5 * dt * dt * a / s->dx;         /* x_{n+1}    */
            p->vx[i] = vnew;
            p->abar[i] = 0.5 * (p->abar[i] + a);                 /* abar_n     */
            int e = boundary(s, &p->xi[i]);
            if (e >= 0) {
                s->led.absorbed_n[k][e]++;
                s->led.absorbed_K[k][e] += kin(p, p->vx[i], p->vy[i], p->vz[i]);
                remove_particle(p, i);
                continue;
            }
            ++i;
        }
    }
    if (s->c.collisions) mcc_all(s);
    /* kinetic energy at n+1/2 is taken before the prediction */
    end_ledger(s, 1);
    for (int k = 0; k < 2; ++k) {
        species_t* p = &s->sp[k];
        if (!moves(s, k)) continue;
        double dt = s->c.dt_s * substep(s, k), dt_dx = dt / s->dx;
        int64_t i = 0;
        while (i < p->n) {
            double vt = p->vx[i] + 0.5 * dt * p->abar[i];
            p->vx[i] = vt;
            if (s->cw) move_nonuniform(s, &p->xi[i], vt * dt);
            else p->xi[i] += vt * dt_dx;
            int e = boundary(s, &p->xi[i]);
            if (e >= 0) {
                double vh1 = vt - 0.5 * dt * p->abar[i];
                double kk = kin(p, vh1, p->vy[i], p->vz[i]);
                s->led.absorbed_n[k][e]++;
                s->led.absorbed_K[k][e] += kk;
                s->led.K_after[k] -= kk;
                remove_particle(p, i);
                continue;
            }
            ++i;
        }
    }
    s->step++;
}

int orc_implicit_startup(orc_sim* s)
{
    for (int k = 0; k < 2; ++k) {
        species_t* p = &s->sp[k];
        double dt = s->c.dt_s * substep(s, k), dt_dx = dt / s->dx;
        int64_t i = 0;
        while (i < p->n) {
            p->abar[i] = 0.0;
            if (s->cw) move_nonuniform(s, &p->xi[i], p->vx[i] * dt);
            else p->xi[i] += p->vx[i] * dt_dx;
            if (boundary(s, &p->xi[i]) >= 0) { remove_particle(p, i); continue; }
            ++i;
        }
    }
    return 0;
}

int orc_step(orc_sim* s, int64_t n)
{
    for (int64_t k = 0; k < n; ++k) {
        if (s->c.scheme == ORC_IMPLICIT) step_implicit(s);
        else step_explicit(s);
    }
    return 0;
}

int orc_step_with_field(orc_sim* s, const double* E)
{
    s->ext_E = E;
    orc_step(s, 1);
    s->ext_E = NULL;
    return 0;
}

int64_t orc_count(const orc_sim* s, int32_t sp) { return s->sp[sp].n; }
int64_t orc_step_index(const orc_sim* s) { return s->step; }

void orc_get_species(const orc_sim* s, int32_t sp, double* xi, double* vx, double* vy,
                     double* vz, double* abar, uint64_t* id, int64_t* wait)
{
    const species_t* p = &s->sp[sp];
    for (int64_t i = 0; i < p->n; ++i) {
        if (xi) xi[i] = p->xi[i];
        if (vx) vx[i] = p->vx[i];
        if (vy) vy[i] = p->vy[i];
        if (vz) vz[i] = p->vz[i];
        if (abar) abar[i] = p->abar[i];
        if (id) id[i] = p->id[i];
        if (wait) wait[i] = p->wait[i];
    }
}

void orc_get_fields(const orc_sim* s, double* rho, double* phi, double* E, double* chi,
                    double* Qe, double* Qi, double* cnt_e, double* cnt_i)
{
    int32_t N = s->c.n_cells;
    size_t nb = sizeof(double) * ((size_t)N + 1), cb = sizeof(double) * (size_t)N;
    if (rho) memcpy(rho, s->rho, nb);
    if (phi) memcpy(phi, s->phi, nb);
    if (E) memcpy(E, s->E, cb);
    if (chi) memcpy(chi, s->chi, cb);
    if (Qe) memcpy(Qe, s->Q[0], nb);
    if (Qi) memcpy(Qi, s->Q[1], nb);
    if (cnt_e) memcpy(cnt_e, s->cnt[0], cb);
    if (cnt_i) memcpy(cnt_i, s->cnt[1], cb);
}

void orc_get_ledger(const orc_sim* s, orc_ledger* out) { *out = s->led; }

void orc_get_heating(const orc_sim* s, double* he, double* hi)
{
    size_t cb = sizeof(double) * (size_t)s->c.n_cells;
    if (he) memcpy(he, s->heat[0], cb);
    if (hi) memcpy(hi, s->heat[1], cb);
}
