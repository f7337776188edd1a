// Device helpers shared by the kernels of the library: the counter-based
// generator, sampling helpers, position normalisation and workgroup-wide
// reductions and scans (kBlock threads).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"
#include "pic_device.hpp"

namespace pic {

// Pointers into device memory in the global address space: loads and stores
// through them compile to global (not flat) instructions, which do not tie up
// the LDS counter and keep independent loads in flight together.
#define PIC_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ PIC_GLOBAL T* gp(T* p)
{
    return (PIC_GLOBAL T*)p;
}

// Workgroup barrier that orders LDS only: it waits for the wavefront's LDS
// operations but not for its outstanding global stores (which only later
// kernels read), so a barrier after a burst of stores does not stall on
// their acknowledgements.  Global data shared inside a workgroup must not be
// handed over through it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A pointer known to be the same in every lane, moved to scalar registers.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T*)(((uint64_t)hi << 32) | lo);
}

// Load / store at a 32-bit byte offset from a global base held in scalar
// registers: one address form (scalar base + vector offset) instead of 64-bit
// vector address arithmetic per access.  Arrays addressed this way stay below
// 4 GiB.
template <class T>
__device__ __forceinline__ T ldg(const PIC_GLOBAL T* base, uint32_t byte_off)
{
    return *(const PIC_GLOBAL T*)((const PIC_GLOBAL char*)base + byte_off);
}
template <class T>
__device__ __forceinline__ void stg(PIC_GLOBAL T* base, uint32_t byte_off, T v)
{
    *(PIC_GLOBAL T*)((PIC_GLOBAL char*)base + byte_off) = v;
}
// The same with the non-temporal cache policy (scattered accesses that touch
// a small part of a line).
template <class T>
__device__ __forceinline__ T ldg_nt(const PIC_GLOBAL T* base, uint32_t byte_off)
{
    return __builtin_nontemporal_load((const PIC_GLOBAL T*)((const PIC_GLOBAL char*)base + byte_off));
}
template <class T>
__device__ __forceinline__ void stg_nt(PIC_GLOBAL T* base, uint32_t byte_off, T v)
{
    __builtin_nontemporal_store(v, (PIC_GLOBAL T*)((PIC_GLOBAL char*)base + byte_off));
}

// The collision record of a particle: id (x, y), vy (z), vz (w).
__device__ __forceinline__ uint64_t rec_id(u32x4 r) { return (uint64_t)r.x | ((uint64_t)r.y << 32); }
__device__ __forceinline__ float rec_vy(u32x4 r) { return __uint_as_float(r.z); }
__device__ __forceinline__ float rec_vz(u32x4 r) { return __uint_as_float(r.w); }
__device__ __forceinline__ u32x4 make_rec(uint64_t id, float vy, float vz)
{
    u32x4 r;
    r.x = (uint32_t)id;
    r.y = (uint32_t)(id >> 32);
    r.z = __float_as_uint(vy);
    r.w = __float_as_uint(vz);
    return r;
}

// relaxed device-scope atomic add through a global pointer
template <class T>
__device__ __forceinline__ T gatomic_add(PIC_GLOBAL T* p, T v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the round keys bumped by the Weyl constants.
// The key is per case (uniform across the wavefront), so the key schedule
// stays in scalar registers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// odd multiple of 2^-24 in (0,1), exact in fp32
__device__ __forceinline__ float u01(uint32_t r)
{
    return (float)((r >> 9) * 2u + 1u) * 5.9604644775390625e-08f;
}

__device__ __forceinline__ void iso_dir(float ua, float ub, float& dx, float& dy, float& dz)
{
    const float ct = 1.0f - 2.0f * ua;
    const float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
    float sp, cp;
    sincospif(2.0f * ub, &sp, &cp);
    dx = st * cp;
    dy = st * sp;
    dz = ct;
}

__device__ __forceinline__ void box_muller(float ua, float ub, float& n1, float& n2)
{
    const float r = sqrtf(-2.0f * logf(ua));
    float sp, cp;
    sincospif(2.0f * ub, &sp, &cp);
    n1 = r * cp;
    n2 = r * sp;
}

__device__ __forceinline__ uint64_t child_id(uint64_t parent, uint32_t step, uint32_t sp_child,
                                             uint32_t k0, uint32_t k1)
{
    const uint4 r = philox((uint32_t)parent, (uint32_t)(parent >> 32), step,
                           (sp_child << 28) | 0x0FFFFFFu, k0, k1);
    return ((uint64_t)r.x | ((uint64_t)r.y << 32)) | (1ull << 63);
}

// ---------------------------------------------------------------------------
// Particle cell word: bit 31 set (negative) for an empty slot, else the cell
// index in bits 0..12 and the null-collision waiting-time field in bits
// 13..30: 17 bits of expiry and the capped flag (PIC_WAIT_CAPPED).
//
// The field holds the value of the species' clock at which the particle's
// count of non-candidate steps reaches zero, modulo 2^17: count =
// (expiry - clock) mod 2^17.  The clock counts the steps in which the
// species takes collision trials (every step; subcycled ions every K-th,
// n / K; none, and the clock stands at 0, when the species has no
// collision process or collisions are off).  The count thus falls by one
// per trial step without the word being rewritten, and a particle's word
// changes only when its cell does or at a candidacy.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint32_t wait_count(uint32_t field, uint32_t clock)
{
    return (field - clock) & PIC_WAIT_MAX;
}
// The field of a count | capped code valid at the given clock.
__host__ __device__ inline uint32_t wait_field(uint32_t clock, uint32_t code)
{
    return ((clock + (code & PIC_WAIT_MAX)) & PIC_WAIT_MAX) | (code & PIC_WAIT_CAPPED);
}
// The species' clock of the first step at or after `step` in which it takes
// trials (trials: whether it takes any).
__host__ __device__ inline uint32_t clock_from(long long step, int ksub, bool trials)
{
    if (!trials) return 0u;
    return (uint32_t)(ksub > 1 ? (step + ksub - 1) / ksub : step);
}
constexpr int kCellBits = 13;
constexpr int32_t kCellMask = (1 << kCellBits) - 1;

__device__ __forceinline__ int32_t pack_cell(int c, uint32_t wait)
{
    return c | (int32_t)(wait << kCellBits);
}
__device__ __forceinline__ int cell_of(int32_t word) { return word >= 0 ? (word & kCellMask) : -1; }
__device__ __forceinline__ uint32_t wait_of(int32_t word) { return (uint32_t)word >> kCellBits; }

// Waiting time W ~ Geo0(P_null) by inversion, W = floor(ln u / ln(1 - P_null)),
// in float64 (inv = 1 / ln(1 - P_null); 0 when P_null >= 1, giving W = 0).
__device__ __forceinline__ double geo0(uint32_t r, double inv)
{
    return floor(log((double)u01(r)) * inv);
}
__device__ __forceinline__ uint32_t wait_encode(double W)
{
    return W > (double)PIC_WAIT_MAX ? (PIC_WAIT_MAX | PIC_WAIT_CAPPED) : (uint32_t)W;
}

// ---------------------------------------------------------------------------
// block-wide helpers (kBlock threads)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Total of a uint32 over the 64 lanes, through DPP row shifts and row
// broadcasts (no LDS traffic).  Must be called with every lane active.
__device__ __forceinline__ unsigned wave_total_u32(unsigned v)
{
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);  // row_shr:8
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false); // row_bcast:15
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false); // row_bcast:31
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Sum over a workgroup of NT threads; every thread gets the result.  red
// holds NT/64 values.
template <typename T, int NT = kBlock>
__device__ __forceinline__ T block_sum(T v, T* red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    lds_barrier();
    if (lane == 0) red[wave] = v;
    lds_barrier();
    T r = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) r += red[w];
    return r;
}

// inclusive prefix sum of a[0..n) in LDS by NT threads, fixed summation order
template <typename T, int NT = kBlock>
__device__ void block_scan(T* a, int n, T* red)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (n + NT - 1) / NT;
    const int lo = min(tid * per, n), hi = min(lo + per, n);
    T loc = 0;
    for (int i = lo; i < hi; ++i) loc += a[i];
    T inc = loc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    lds_barrier();
    if (lane == 63) red[wave] = inc;
    lds_barrier();
    T run = inc - loc;
    for (int w = 0; w < wave; ++w) run += red[w];
    for (int i = lo; i < hi; ++i) {
        run += a[i];
        a[i] = run;
    }
    lds_barrier();
}

// "no cell touched" marker of the range trackers; far from INT_MAX so that
// lo + threadIdx.x cannot overflow
constexpr int kNoCell = 0x3fffffff;

__device__ __forceinline__ void range_note(int& lo, int& hi, int c)
{
    lo = min(lo, c);
    hi = max(hi, c);
}

// Normalise (cell, off) after a move: off in [0,1), an offset that rounds to
// 1.0f moves to the next cell.
__device__ __forceinline__ void renorm(int& c, float& o)
{
    const float fl = floorf(o);
    c += (int)fl;
    o -= fl;
    if (o >= 1.0f) {
        o = 0.0f;
        c += 1;
    }
}

// D1 prediction from x_{n+1} = (c, o) with v_{n+1/2} and abar_n (cells per
// step): v~ = v + abar/2, x~ = x + v~.  One rounding per operation, so that
// k_step and k_collide reproduce the same prediction bit for bit.  Returns v~.
//
// kf: the species' time step in units of dt (K for subcycled ions, else 1):
// v~ = v + kf abar / 2, x~ = x + kf v~.
__device__ __forceinline__ float predict(int& c, float& o, float vn, float abn, float kf = 1.0f)
{
    const float vst = fmaf(0.5f * kf, abn, vn);
    o = __fadd_rn(o, kf * vst);
    renorm(c, o);
    return vst;
}

// A move by d (units of the reference width L/N) on a nonuniform grid with
// r[c] = (L/N) / w_c, where run[c] holds the first (low 16 bits) and last
// (high 16 bits) cell of the run of equal widths that contains c.  Inside a
// run the move is the uniform one (offset + d r_c, whole cells carried into
// the index); at the end of a run the rest of the move continues in the
// next run.  Past an electrode the walk stops with the cell index -1 or N,
// which the boundary rule absorbs.  Each run is visited at most once.  One
// rounding per operation, so that every kernel reproduces the same walk bit
// for bit.
template <class RP, class UP>
__device__ __forceinline__ void walk(int& c, float& o, float d, RP r, UP run, int N)
{
    if (d >= 0.0f) {
        for (;;) {
            const float rc = r[c];
            const float x = fmaf(d, rc, o);
            if (x < 1.0f) {
                o = x;
                return;
            }
            const int hi = (int)(run[c] >> 16);
            const float fl = floorf(x);
            if ((float)(hi - c) >= fl) {   // ends inside the run
                c += (int)fl;
                o = x - fl;
                if (o >= 1.0f) {
                    o = 0.0f;
                    c += 1;
                }
                return;
            }
            // to the right end of the run, then on into the next one
            d = __fsub_rn(d, __fdiv_rn(__fsub_rn((float)(hi + 1 - c), o), rc));
            c = hi + 1;
            o = 0.0f;
            if (c >= N || d <= 0.0f) return;
        }
    }
    for (;;) {
        const float rc = r[c];
        const float x = fmaf(d, rc, o);
        if (x >= 0.0f) {
            if (x >= 1.0f) {   // a rest too small to leave the right edge
                ++c;
                o = 0.0f;
            } else {
                o = x;
            }
            return;
        }
        const int lo = (int)(run[c] & 0xFFFFu);
        const float fl = floorf(x);   // negative
        if ((float)(lo - c) <= fl) {   // ends inside the run
            c += (int)fl;
            o = x - fl;
            if (o >= 1.0f) {
                o = 0.0f;
                c += 1;
            }
            return;
        }
        // to the left end of the run, then on into the previous one
        d = __fadd_rn(d, __fdiv_rn(__fadd_rn((float)(c - lo), o), rc));
        c = lo - 1;
        o = 1.0f;   // the right edge of the cell entered
        if (c < 0) return;
        if (d >= 0.0f) {   // the move ended on the edge
            c = lo;
            o = 0.0f;
            return;
        }
    }
}

// The D1 prediction on a nonuniform grid (the walk in place of renorm).
template <class RP, class UP>
__device__ __forceinline__ float predict_nu(int& c, float& o, float vn, float abn, RP r, UP run,
                                            int N, float kf = 1.0f)
{
    const float vst = fmaf(0.5f * kf, abn, vn);
    walk(c, o, kf * vst, r, run, N);
    return vst;
}

// Flag in the waiting-time field of a listed candidate's word (its count is
// zero): k_step deposited the candidate's prediction without a collision.
constexpr uint32_t kPredDeposited = 1u;

}  // namespace pic
