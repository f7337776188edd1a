// Weighting and interpolation shared by the particle pass and the set-up
// deposit: the gathers of Eq. (3) (m = 1 own cell, m = 2 linear of the
// half-grid field, MC linear of the nodal field), the packed linear weight of
// Eq. (2), the quadratic weights and deposit of Eq. (2) with m = 2, and its
// moment form for the implicit scheme (node charges and susceptibility).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"
#include "pic_common.hpp"
#include "pic_device.hpp"

namespace pic {

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

// The same on a nonuniform grid (electrodes) with r[c] = (L/N) / w_c: the
// centred difference of the potential over the node's two cells, i.e. the
// width-weighted mean (w_{g-1} E_{g-1} + w_g E_g) / (w_{g-1} + w_g) =
// (r_g E_{g-1} + r_{g-1} E_g) / (r_{g-1} + r_g).
__device__ __forceinline__ float nodal_field_nu(const PIC_GLOBAL float* eh,
                                                const PIC_GLOBAL float* r, int N, int g)
{
    if (g == 0) return eh[0];
    if (g == N) return eh[N - 1];
    return (r[g] * eh[g - 1] + r[g - 1] * eh[g]) / (r[g - 1] + r[g]);
}

__device__ __forceinline__ unsigned long long packw(float o)
{
    return kCountOne + (unsigned long long)__float2uint_rn(o * 16777216.0f);
}

// The quadratic deposit of the implicit scheme with m = 2, in moment form.
// Its susceptibility (Sec. II, degree reading): displacing a particle moves,
// through the quadratic deposit, the flux S_1(x_p - x_h) d_p through centre
// h, and the D1 correction d_p follows the linear gather of the half-grid
// field, so the exact operator is proportional to sum_p S_1(x_p - x_h)
// S_1(x_p - x_h'); the solve takes its row sums.  A particle with nearest
// node i lies between centres i-1 and i, at fraction t = 1/2 + d towards i.
// Words:
// per nearest node i (the dual word of the susceptibility), word A[i] =
// (particles of cell i) << 40 | sum of their weights P0 to node i-1, and
// B[i] = (particles of cell i-1) << 40 | sum of the weights P2 to node i+1
// (P0, P2 of quad_weights; a periodic node N is node 0).  From these the
// solve forms the same node charges as the deposit of deposit_quad, the cell
// counts, and the susceptibility fractions (t = 1/2 + (P2 - P0) 2^-24, t^2 =
// 2 P2 2^-24, (1 - t)^2 = 2 P0 2^-24 per particle).  sorted: the lanes of a
// cell-sorted species share at most two nodes; their words are summed
// across the wavefront first (called by whole wavefronts then).
// L0, L2 (nonuniform grid, else null): the P0 and P2 sums of the particles
// left of their nearest node.
__device__ __forceinline__ void deposit_moments(unsigned long long* A, unsigned long long* B,
                                                bool want, int c, float o, int N, bool periodic,
                                                int& lo, int& hi, bool sorted = false,
                                                unsigned long long* L0 = nullptr,
                                                unsigned long long* L2 = nullptr)
{
    uint32_t w[3] = {0u, 0u, 0u};
    int i = c;
    if (want) i = quad_weights(c, o, w);
    if (periodic && i == N) i = 0;
    const bool left = o >= 0.5f;   // the particle lies left of node i (in cell i-1)
    if (sorted) {
        const unsigned long long m = __ballot(want);
        if (m == 0ull) return;
        const int lane = threadIdx.x & 63;
        const int ia = __builtin_amdgcn_readlane(i, __ffsll((long long)m) - 1);
        const unsigned long long ma = __ballot(want && i == ia);
        const unsigned long long mb = m & ~ma;
        const int ib = mb ? __builtin_amdgcn_readlane(i, __ffsll((long long)mb) - 1) : ia;
        if (__ballot(want && i != ia && i != ib) == 0ull) {
            const unsigned long long ml = __ballot(want && left);
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const unsigned long long mg = g == 0 ? ma : mb;
                if (mg == 0ull) continue;
                // at most 64 * 2^23 per sum
                const bool mine = ((mg >> lane) & 1ull) != 0ull;
                const unsigned t0 = wave_total_u32(mine ? w[0] : 0u);
                const unsigned t2 = wave_total_u32(mine ? w[2] : 0u);
                unsigned l0 = 0u, l2 = 0u;
                if (L0) {
                    l0 = wave_total_u32(mine && left ? w[0] : 0u);
                    l2 = wave_total_u32(mine && left ? w[2] : 0u);
                }
                if (lane == __ffsll((long long)mg) - 1) {
                    const int ig = g == 0 ? ia : ib;
                    atomicAdd(&A[ig], (unsigned long long)__popcll(mg & ~ml) * kCountOne + t0);
                    atomicAdd(&B[ig], (unsigned long long)__popcll(mg & ml) * kCountOne + t2);
                    if (L0) {
                        if (l0) atomicAdd(&L0[ig], (unsigned long long)l0);
                        if (l2) atomicAdd(&L2[ig], (unsigned long long)l2);
                    }
                    range_note(lo, hi, ig);
                }
            }
            return;
        }
    }
    if (!want) return;
    atomicAdd(&A[i], (left ? 0ull : kCountOne) + (unsigned long long)w[0]);
    atomicAdd(&B[i], (left ? kCountOne : 0ull) + (unsigned long long)w[2]);
    if (L0 && left) {
        atomicAdd(&L0[i], (unsigned long long)w[0]);
        atomicAdd(&L2[i], (unsigned long long)w[2]);
    }
    range_note(lo, hi, i);
}

}  // namespace pic
