// Host runtime and C-ABI of the EC PIC/MCC hot path (see include/pic.h).
//
// Owns all device memory of a context: per case and species a structure-of-
// arrays particle store (two copies for the compaction), the fixed-point
// deposit accumulators, fields, per-case tables and counters.  Launches one
// k_step per scheme group per step, and the compaction every sort_every steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "pic.h"
#include "pic_common.hpp"
#include "pic_device.hpp"

namespace pic {
template <int SCHEME, bool DIAG, bool GT, bool DUAL, bool PLAIN>
__global__ void k_step(Params P);
template <int SCHEME, bool DIAG, bool DUAL, bool PLAIN>
__global__ void k_collide(Params P);
__global__ void k_init_species(Params P, double vscale0, double vscale1);
__global__ void k_compact_hist(Params P, uint32_t* hist_all, const int64_t* hist_off);
__global__ void k_compact_scan(Params P, uint32_t* hist_all, uint32_t* cursor_all,
                               const int64_t* hist_off);
__global__ void k_compact_scatter(Params P, uint32_t* cursor_all, const int64_t* hist_off);
__global__ void k_compact_finish(Params P);
__global__ void k_deposit(Params P);
__global__ void k_solve(Params P);
template <bool kDual, bool kPlain>
__global__ void k_finalize(Params P, int sample);
}  // namespace pic

using namespace pic;

namespace {

constexpr double QE = 1.602176634e-19;
constexpr double EPS0 = 8.8541878128e-12;
constexpr int kCellWordBits = 13;   // cell index bits of the device cell word
constexpr double KB = 1.380649e-23;
constexpr double ME_LIMIT = 1e-27;  // species lighter than this are "electron-like"

struct HostCase {
    pic_case_config cfg;
    double scale[2];        // n_g (dx/dt) / nu_max per species (collision tables)
    double pnull[2] = {0.0, 0.0};   // null-collision candidate probability per step
    double q[2], m[2], w[2];
    int64_t cap[2];
    int64_t n0[2];
    double vscale;          // (m/s) -> cells/step
    std::vector<double> cell_w;   // nonuniform grid: widths (m); empty if uniform
    // float64 values of the per-species collision constants that the float
    // path stores as float32 (for the plain FP64 form): eps_unit, opal_B,
    // recoil2, vth_neutral, vth_newion, t_scale, t_off, t_max, thr_v2[4]
    double c64[2][12];
    size_t hist_off[2];
    // device allocations owned by the case
    std::vector<void*> allocs;
};

struct FP64Ref;  // plain FP64 GPU form (pic_fp64.hip)

// Timing events around the particle and collision kernels: pairs (start,
// stop) in launch order, with the kernel each pair brackets.
struct EventPool {
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;          // 0: k_step, 1: k_collide
    int used = 0;
};

// One sort period (sort_every steps and the compaction after them) captured
// into a HIP graph.  Its timing events are recorded by event nodes, so after
// several replays they hold the last replay's times.
struct PeriodGraph {
    hipGraphExec_t exec = nullptr;
    EventPool ev;
    int period = 0;
};

}  // namespace

struct pic_ctx {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // a batch holding both schemes runs the implicit group's kernels, and
    // the finalizer of its cases, on a second stream (the groups touch
    // disjoint cases); the streams are joined before a compaction, a step
    // on one stream, a graph replay and the end of a call
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool forked = false;   // stream2 has work that the context's stream has not joined
    bool nt_store = false;   // store policy of k_collide (pic_set_store_policy)
    bool failed = false;
    std::string err;
    int n_cases = 0;
    std::vector<HostCase> hc;
    std::vector<Case> cases_h;      // host mirror (pointers valid after set-up)
    Case* d_cases = nullptr;
    State* d_state = nullptr;
    Work* d_work = nullptr;
    double* d_pd = nullptr;        // workgroup partials (field-major)
    unsigned* d_pu = nullptr;
    int32_t* d_cand_n = nullptr;    // candidates listed by each workgroup
    uint32_t* d_hist = nullptr;
    uint32_t* d_cursor = nullptr;
    int64_t* d_hist_off = nullptr;
    std::vector<Work> work;
    int n_blocks = 0;
    int grp_off[2] = {0, 0}, grp_cnt[2] = {0, 0};   // explicit, implicit workgroups
    std::vector<CollideWork> cwork;                 // k_collide work table
    int cgrp_off[2] = {0, 0}, cgrp_cnt[2] = {0, 0};
    CollideWork* d_cwork = nullptr;
    size_t grp_slds[2][2] = {{0, 0}, {0, 0}};   // k_step LDS of a group ([diag])
    bool grp_gt[2] = {false, false};   // k_step reads the grid tables from global memory
    bool grp_dual[2] = {false, false};   // a case of the group has the m = 2 moment words
    bool grp_plain[2] = {true, true};    // every case of the group: EC gather, uniform grid
    size_t grp_clds[2] = {0, 0};                // k_collide LDS of a group
    size_t dep_lds_max = 0;                     // k_deposit LDS over all cases
    bool any_dual = false;
    int maxN = 0;
    int tile = 8192;
    int sort_every = 64;
    int diag_every = 0;
    int64_t since_sort = 0;
    int64_t steps_taken = 0;
    EventPool ev;                  // events of host-launched steps
    double last_ms = 0.0;
    int64_t last_launches = 0;
    double last_ms_coll = 0.0;
    int64_t last_launches_coll = 0;
    int timing_every = 1;          // steps between timed steps (0: none)
    bool use_graph = false;
    PeriodGraph graph;             // one sort period, captured on first use
    void* fp64 = nullptr;          // FP64 reference form (pic_fp64.hip)
    std::vector<void*> allocs;     // context-level allocations
    std::vector<std::vector<double>> sigma[2];   // float64 copy of the input tables
    size_t hist_total = 0;         // compaction histogram words (all cases, species)
    int device = 0;                // HIP device current at pic_init
    void* fixed_scratch = nullptr; // this device's address of the fixed scratch array
    // pic_step_noalloc: the step's scratch (workgroup partials, candidate
    // counts, compaction histograms and cursors) is taken from the fixed
    // array while `use_fixed` is set
    bool use_fixed = false;
    double* fx_pd = nullptr;
    unsigned* fx_pu = nullptr;
    int32_t* fx_cand_n = nullptr;
    uint32_t* fx_hist = nullptr;
    uint32_t* fx_cursor = nullptr;
};

// Fixed scratch of pic_step_noalloc: the per-step scratch of the kernels
// (ledger partial rows and candidate counts of every k_step workgroup, the
// compaction's bucket histograms and cursors) for callers that cannot
// allocate.  One array per device, held until the process ends; host code
// reaches it only through the address hipGetSymbolAddress gives on that
// device (resolve_fixed_scratch).
constexpr size_t kFixedScratchBytes = (size_t)2 << 20;
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void* g_fixed_ptr[kMaxDevices] = {};

__global__ void k_fill_u32(uint32_t* p, uint32_t n, uint32_t v)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = v;
}

int fail(pic_ctx* c, int code, const std::string& msg)
{
    if (c) {
        c->err = msg;
        if (code == PIC_E_DEVICE || code == PIC_E_STATE) c->failed = true;
    }
    return code;
}

#define HIPCHK(ctx, expr)                                                              \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(ctx, PIC_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// inside pic_init: report, free the partial context and return
#define INITCHK(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return bail(fail(c, PIC_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_))); \
    } while (0)

template <typename T>
int dalloc(pic_ctx* c, std::vector<void*>& list, T** p, size_t n)
{
    void* q = nullptr;
    size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    if (hipMalloc(&q, bytes) != hipSuccess) return fail(c, PIC_E_NOMEM, "hipMalloc failed");
    if (hipMemset(q, 0, bytes) != hipSuccess) {
        (void)hipFree(q);
        return fail(c, PIC_E_DEVICE, "hipMemset failed");
    }
    list.push_back(q);
    *p = (T*)q;
    return PIC_OK;
}

// The address of this device's fixed scratch array, resolved once per device
// (with that device current) and kept for every later context on it.
int resolve_fixed_scratch(pic_ctx* c)
{
    int dev = 0;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(c, PIC_E_DEVICE, "device index beyond the fixed-scratch table");
    std::lock_guard<std::mutex> lock(g_fixed_mu);
    if (!g_fixed_ptr[dev]) {
        void* ptr = nullptr;
        HIPCHK(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_fixed_ptr[dev] = ptr;
    }
    c->device = dev;
    c->fixed_scratch = g_fixed_ptr[dev];
    return PIC_OK;
}

size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

// Dynamic LDS of k_step: field[N+1] float | dep[N+1] u64 | (m = 2 implicit:
// susceptibility words[N+1] u64) | (DIAG: heat[N] float | eedf[kEedfBins] u32).
size_t step_lds(int N, bool diag, bool dual, bool nu, bool tables = true)
{
    return step_lds_layout(N, diag, dual, nu, tables).total;
}

// A group with an m = 2 implicit case on a nonuniform grid launches the
// k_step variant that reads the width ratios and runs from global memory.
bool global_tables(bool dual, bool nu)
{
    return dual && nu;
}

size_t collide_lds(int N, bool dual, bool nu)
{
    return collide_lds_layout(N, dual, nu).total;
}

// k_deposit: node words dep[N+1] | (dual) susceptibility words [N+1] |
// (dual, nonuniform) left-side sums 2 x [N+1]
size_t deposit_lds(int N, bool dual, bool nu)
{
    return 8 * ((size_t)N + 1) * (dual ? (nu ? 4 : 2) : 1);
}

// the most dynamic LDS one workgroup may hold
constexpr size_t kLdsMax = 160 * 1024;

// the largest LDS any kernel of one case asks for
size_t case_lds(int N, bool dual, bool nu)
{
    return std::max(std::max(step_lds(N, true, dual, nu, !global_tables(dual, nu)),
                             collide_lds(N, dual, nu)),
                    deposit_lds(N, dual, nu));
}

// k_finalize / k_solve: rho prefix S[N+1], chi per cell X[N], chi per node
// Y[N+1] (fp64), and a reduction slot
size_t fin_lds(int N)
{
    return 24 * ((size_t)N + 1) + 16;
}

// Null-collision bound: n_g max over table intervals of
// max(sigma_T(e_i), sigma_T(e_{i+1})) v(e_{i+1}), v = sqrt(2 e eps / m).
double nu_max(const std::vector<const pic_xsec*>& pr, double ng, double mass)
{
    if (pr.empty()) return 0.0;
    const pic_xsec* a = pr[0];
    double best = 0.0;
    for (int32_t i = 0; i + 1 < a->n; ++i) {
        double sl = 0.0, sr = 0.0;
        for (const pic_xsec* p : pr) {
            sl += p->sigma_m2[i];
            sr += p->sigma_m2[i + 1];
        }
        double er = a->e0_eV + (double)(i + 1) * a->de_eV;
        double v = std::sqrt(2.0 * QE * (er > 0.0 ? er : 0.0) / mass);
        best = std::max(best, std::max(sl, sr) * v);
    }
    return ng * best;
}

uint32_t candidate_threshold(double pnull)
{
    // number of k in [0, 2^23) with (2k+1) 2^-24 < pnull
    double t = (pnull * 16777216.0 - 1.0) / 2.0;
    double c = std::ceil(t);
    if (c < 0.0) c = 0.0;
    if (c > 8388608.0) c = 8388608.0;
    return (uint32_t)c;
}

// k_collide rounds: candidates per thread aimed at, and the most rounds
// (8 and 16 measured slower than 32 on a batch of high-pressure cases, where
// most particles are candidates; lists of a few % of a tile take one round)
constexpr double kCandPerThread = 64.0;
constexpr int kMaxRounds = 32;

int build_work(pic_ctx* c)
{
    c->work.clear();
    c->cwork.clear();
    for (int g = 0; g < 2; ++g) {
        c->grp_off[g] = (int)c->work.size();
        c->grp_slds[g][0] = c->grp_slds[g][1] = 0;
        c->grp_clds[g] = 0;
        c->grp_gt[g] = false;
        c->grp_dual[g] = false;
        c->grp_plain[g] = true;
        for (int k = 0; k < c->n_cases; ++k) {
            const HostCase& h = c->hc[k];
            if (h.cfg.scheme != g) continue;
            const bool dk = dual_chi(h.cfg.scheme, h.cfg.gather);
            c->grp_gt[g] = c->grp_gt[g] || global_tables(dk, !h.cell_w.empty());
            c->grp_dual[g] = c->grp_dual[g] || dk;
            c->grp_plain[g] = c->grp_plain[g] && h.cfg.gather == PIC_GATHER_EC && h.cell_w.empty();
        }
        for (int k = 0; k < c->n_cases; ++k) {
            HostCase& h = c->hc[k];
            if (h.cfg.scheme != g) continue;
            Case& C = c->cases_h[k];
            C.first_block = (int)c->work.size();
            for (int s = 0; s < 2; ++s) {
                int nb = (int)std::max<int64_t>(1, (h.cap[s] + c->tile - 1) / c->tile);
                for (int b = 0; b < nb; ++b) c->work.push_back(Work{k, s, b, nb});
            }
            C.n_blocks = (int)c->work.size() - C.first_block;

            // each workgroup lays its LDS out for its own case: the launch
            // takes the largest
            const int Nk = h.cfg.n_cells;
            const bool dk = dual_chi(h.cfg.scheme, h.cfg.gather), nk = !h.cell_w.empty();
            for (int d = 0; d < 2; ++d)
                c->grp_slds[g][d] =
                    std::max(c->grp_slds[g][d], step_lds(Nk, d == 1, dk, nk, !c->grp_gt[g]));
            c->grp_clds[g] = std::max(c->grp_clds[g], collide_lds(Nk, dk, nk));
        }
        c->grp_cnt[g] = (int)c->work.size() - c->grp_off[g];
    }
    c->n_blocks = (int)c->work.size();
    // k_collide: for every k_step workgroup that can list candidates, as
    // many workgroups (rounds) as its expected list needs at about
    // kCandPerThread candidates per thread; they add their collision terms
    // to the ledger row of that k_step workgroup.  The workgroups of a group
    // are ordered by their expected candidates per thread, largest first, so
    // that the long rounds of dense lists start first and the short ones
    // fill in behind them.
    for (int g = 0; g < 2; ++g) {
        c->cgrp_off[g] = (int)c->cwork.size();
        std::vector<std::pair<double, CollideWork>> order;
        for (int k = 0; k < c->n_cases; ++k) {
            HostCase& h = c->hc[k];
            if (h.cfg.scheme != g) continue;
            Case& C = c->cases_h[k];
            for (int b = C.first_block; b < C.first_block + C.n_blocks; ++b) {
                const Work& w = c->work[b];
                const double p = h.cfg.collisions ? h.pnull[w.s] : 0.0;
                if (!(p > 0.0)) continue;
                const double per_wg = (double)std::min<int64_t>(c->tile, h.cap[w.s]);
                const int rounds = (int)std::min<double>(
                    kMaxRounds, std::max(1.0, std::ceil(p * per_wg / (kBlock * kCandPerThread))));
                const double load = p * per_wg / (rounds * (double)kBlock);
                for (int r = 0; r < rounds; ++r)
                    order.emplace_back(load, CollideWork{b, r, rounds, 0, w});
            }
        }
        std::stable_sort(order.begin(), order.end(),
                         [](const std::pair<double, CollideWork>& a,
                            const std::pair<double, CollideWork>& b) { return a.first > b.first; });
        for (const auto& e : order) c->cwork.push_back(e.second);
        c->cgrp_cnt[g] = (int)c->cwork.size() - c->cgrp_off[g];
    }
    return PIC_OK;
}

int upload_work(pic_ctx* c)
{
    if (c->d_work) (void)hipFree(c->d_work);
    if (c->d_pd) (void)hipFree(c->d_pd);
    if (c->d_pu) (void)hipFree(c->d_pu);
    if (c->d_cand_n) (void)hipFree(c->d_cand_n);
    if (c->d_cwork) (void)hipFree(c->d_cwork);
    c->d_work = nullptr;
    c->d_pd = nullptr;
    c->d_pu = nullptr;
    c->d_cand_n = nullptr;
    c->d_cwork = nullptr;
    const size_t nb = c->work.size();
    const size_t ncw = c->cwork.size();
    const size_t rows = nb;   // ledger partial rows: one per k_step workgroup
    HIPCHK(c, hipMalloc(&c->d_work, sizeof(Work) * nb));
    HIPCHK(c, hipMemcpy(c->d_work, c->work.data(), sizeof(Work) * nb, hipMemcpyHostToDevice));
    HIPCHK(c, hipMalloc(&c->d_cwork, sizeof(CollideWork) * std::max<size_t>(ncw, 1)));
    if (ncw)
        HIPCHK(c, hipMemcpy(c->d_cwork, c->cwork.data(), sizeof(CollideWork) * ncw,
                            hipMemcpyHostToDevice));
    HIPCHK(c, hipMalloc(&c->d_pd, sizeof(double) * PD_N * rows));
    HIPCHK(c, hipMemset(c->d_pd, 0, sizeof(double) * PD_N * rows));
    HIPCHK(c, hipMalloc(&c->d_pu, sizeof(unsigned) * PU_N * rows));
    HIPCHK(c, hipMemset(c->d_pu, 0, sizeof(unsigned) * PU_N * rows));
    HIPCHK(c, hipMalloc(&c->d_cand_n, sizeof(int32_t) * nb));
    HIPCHK(c, hipMemset(c->d_cand_n, 0, sizeof(int32_t) * nb));

    return PIC_OK;
}

Params params(pic_ctx* c, int mode)
{
    Params p;
    p.cases = c->d_cases;
    p.state = c->d_state;
    p.work = c->d_work;
    p.pd = c->use_fixed ? c->fx_pd : c->d_pd;
    p.pu = c->use_fixed ? c->fx_pu : c->d_pu;
    p.stride = (int32_t)c->work.size();
    p.n_cases = c->n_cases;
    p.mode = mode;
    p.cand_n = c->use_fixed ? c->fx_cand_n : c->d_cand_n;
    p.cwork = c->d_cwork;
    p.nt_store = c->nt_store ? 1 : 0;

    return p;
}

int compaction(pic_ctx* c)
{
    Params p = params(c, 0);
    size_t l1 = 4 * (size_t)c->maxN, l2 = 8 * (size_t)c->maxN;
    uint32_t* hist = c->use_fixed ? c->fx_hist : c->d_hist;
    uint32_t* cursor = c->use_fixed ? c->fx_cursor : c->d_cursor;
    hipLaunchKernelGGL(k_compact_hist, dim3(c->n_blocks), dim3(kBlock), l1, c->stream, p,
                       hist, (const int64_t*)c->d_hist_off);
    hipLaunchKernelGGL(k_compact_scan, dim3(2 * c->n_cases), dim3(kBlock), l1, c->stream, p,
                       hist, cursor, (const int64_t*)c->d_hist_off);
    hipLaunchKernelGGL(k_compact_scatter, dim3(c->n_blocks), dim3(kBlock), l2, c->stream, p,
                       cursor, (const int64_t*)c->d_hist_off);
    hipLaunchKernelGGL(k_compact_finish, dim3(c->n_cases), dim3(kFinBlock), 0, c->stream, p);
    HIPCHK(c, hipGetLastError());
    c->since_sort = 0;
    return PIC_OK;
}

// Dynamic LDS above the default 64 KiB needs an explicit opt-in per kernel.
// The k_step variant of a scheme group (see k_step: PLAIN, DUAL, GT).
using StepKernel = void (*)(Params);
StepKernel step_kernel(int g, bool diag, bool gt, bool dual, bool plain)
{
    if (g == 0) {
        if (plain) return diag ? k_step<0, true, false, false, true> : k_step<0, false, false, false, true>;
        return diag ? k_step<0, true, false, false, false> : k_step<0, false, false, false, false>;
    }
    if (gt) return diag ? k_step<1, true, true, true, false> : k_step<1, false, true, true, false>;
    if (dual) return diag ? k_step<1, true, false, true, false> : k_step<1, false, false, true, false>;
    if (plain) return diag ? k_step<1, true, false, false, true> : k_step<1, false, false, false, true>;
    return diag ? k_step<1, true, false, false, false> : k_step<1, false, false, false, false>;
}

// The k_collide variant of a scheme group.
StepKernel collide_kernel(int g, bool diag, bool dual, bool plain)
{
    // (the explicit kernel reaches no grid- or weighting-specific code)
    if (g == 0) return diag ? k_collide<0, true, false, false> : k_collide<0, false, false, false>;
    if (dual) return diag ? k_collide<1, true, true, false> : k_collide<1, false, true, false>;
    if (plain) return diag ? k_collide<1, true, false, true> : k_collide<1, false, false, true>;
    return diag ? k_collide<1, true, false, false> : k_collide<1, false, false, false>;
}

int set_lds_limits(pic_ctx* c, size_t need)
{
    if (need <= 65536) return PIC_OK;
    const int v = (int)need;
    const void* ks[] = {(const void*)k_step<0, false, false, false, true>,
                        (const void*)k_step<0, true, false, false, true>,
                        (const void*)k_step<0, false, false, false, false>,
                        (const void*)k_step<0, true, false, false, false>,
                        (const void*)k_step<1, false, false, false, true>,
                        (const void*)k_step<1, true, false, false, true>,
                        (const void*)k_step<1, false, false, false, false>,
                        (const void*)k_step<1, true, false, false, false>,
                        (const void*)k_step<1, false, false, true, false>,
                        (const void*)k_step<1, true, false, true, false>,
                        (const void*)k_step<1, false, true, true, false>,
                        (const void*)k_step<1, true, true, true, false>,
                        (const void*)k_collide<0, false, false, false>,
                        (const void*)k_collide<0, true, false, false>,
                        (const void*)k_collide<1, false, false, true>,
                        (const void*)k_collide<1, true, false, true>,
                        (const void*)k_collide<1, false, false, false>,
                        (const void*)k_collide<1, true, false, false>,
                        (const void*)k_collide<1, false, true, false>,
                        (const void*)k_collide<1, true, true, false>,
                        (const void*)k_compact_scatter, (const void*)k_compact_hist,
                        (const void*)k_compact_scan, (const void*)k_deposit, (const void*)k_solve,
                        (const void*)k_finalize<false, true>,
                        (const void*)k_finalize<false, false>,
                        (const void*)k_finalize<true, false>};
    for (const void* k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, v);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, PIC_E_INVAL, std::string("LDS opt-in of ") + std::to_string(need) +
                                            " bytes refused: " + hipGetErrorString(e));
        }
    }
    return PIC_OK;
}

void destroy_ctx(pic_ctx* c);
void drop_graph(pic_ctx* c);

}  // namespace

// defined in pic_fp64.hip
extern "C" void pic__fp64_free(pic_ctx* ctx);

extern "C" int pic_init(pic_ctx** out, int32_t n_cases, const pic_case_config* cases,
                        const pic_species_init* species, const pic_xsec* xs, int32_t n_xs,
                        void* hip_stream, uint32_t flags)
{
    if (!out) return PIC_E_INVAL;
    *out = nullptr;
    if (n_cases <= 0 || !cases || !species || (n_xs > 0 && !xs) || n_xs < 0) return PIC_E_INVAL;
    pic_ctx* c = new pic_ctx();
    auto bail = [&](int code) {
        if (!c->err.empty()) fprintf(stderr, "pic_init: %s\n", c->err.c_str());
        destroy_ctx(c);
        return code;
    };
    c->n_cases = n_cases;
    c->hc.resize(n_cases);
    c->cases_h.resize(n_cases);
    // ---- validation ----
    for (int k = 0; k < n_cases; ++k) {
        const pic_case_config& g = cases[k];
        if (g.n_cells < 2 || g.n_cells > PIC_MAX_CELLS || !(g.gap_m > 0) || !(g.dt_s > 0) ||
            (g.bc != PIC_BC_DIRICHLET_RF && g.bc != PIC_BC_PERIODIC) ||
            (g.scheme != PIC_EXPLICIT && g.scheme != PIC_IMPLICIT_D1) ||
            (g.gather != PIC_GATHER_EC && g.gather != PIC_GATHER_MC &&
             g.gather != PIC_GATHER_EC2) ||
            g.history_steps < 0 || g.ion_subcycle < 0 || g.ion_subcycle > 4096 ||
            (g.cell_dx_m && g.bc != PIC_BC_DIRICHLET_RF) ||
            g.start_step < 0) {
            fprintf(stderr, "pic_init: case %d: bad configuration\n", k);
            return bail(PIC_E_INVAL);
        }
        if (g.cell_dx_m) {
            double L = 0.0;
            bool ok = true;
            for (int32_t j = 0; j < g.n_cells; ++j) {
                const double wj = g.cell_dx_m[j];
                ok = ok && wj > 0.0 && std::isfinite(wj);
                L += wj;
            }
            if (!ok || !(std::fabs(L - g.gap_m) <= 1e-9 * g.gap_m)) {
                fprintf(stderr, "pic_init: case %d: bad cell widths\n", k);
                return bail(PIC_E_INVAL);
            }
        }
        {
            // (m = 2 implicit on a nonuniform grid: above 4069 cells)
            const size_t need = case_lds(g.n_cells, dual_chi(g.scheme, g.gather),
                                         g.cell_dx_m != nullptr);
            if (need > kLdsMax) {
                fprintf(stderr, "pic_init: case %d: %d cells need %zu bytes of LDS\n", k,
                        g.n_cells, need);
                return bail(PIC_E_INVAL);
            }
        }
        for (int s = 0; s < 2; ++s) {
            const pic_species_init& sp = species[2 * k + s];
            if (sp.n < 0 || sp.capacity < sp.n || sp.capacity > ((int64_t)1 << 28) - 1024 || !(sp.m_kg > 0) ||
                (sp.n > 0 && (!sp.cell || !sp.off || !sp.vx || !sp.vy || !sp.vz || !sp.id))) {
                fprintf(stderr, "pic_init: case %d species %d: bad arrays\n", k, s);
                return bail(PIC_E_INVAL);
            }
        }
        if (g.collisions && (!(g.gas_density_m3 >= 0) || !(g.gas_temp_K > 0) ||
                             !(g.gas_mass_kg > 0) || !(g.opal_B_eV > 0))) {
            fprintf(stderr, "pic_init: case %d: bad gas\n", k);
            return bail(PIC_E_INVAL);
        }
    }
    std::vector<const pic_xsec*> proc[2];
    for (int i = 0; i < n_xs; ++i) {
        const pic_xsec& x = xs[i];
        if (x.species < 0 || x.species > 1 || x.n < 2 || !(x.de_eV > 0) || !x.sigma_m2 ||
            (x.species == 1 && x.kind != PIC_CHARGE_EXCHANGE) ||
            (x.species == 0 && (x.kind < PIC_ELASTIC || x.kind > PIC_IONIZATION)))
            return bail(PIC_E_INVAL);
        proc[x.species].push_back(&x);
    }
    for (int s = 0; s < 2; ++s) {
        if ((int)proc[s].size() > (s == 0 ? kMaxProc : 1)) return bail(PIC_E_INVAL);
        for (const pic_xsec* p : proc[s])
            if (p->n != proc[s][0]->n || p->e0_eV != proc[s][0]->e0_eV ||
                p->de_eV != proc[s][0]->de_eV)
                return bail(PIC_E_INVAL);
    }
    for (int s = 0; s < 2; ++s)
        for (const pic_xsec* p : proc[s])
            c->sigma[s].emplace_back(p->sigma_m2, p->sigma_m2 + p->n);
    // ---- stream ----
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(c, PIC_E_DEVICE, "stream"));
        c->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess)
        return bail(fail(c, PIC_E_DEVICE, "second stream"));
    (void)hipGetLastError();   // start from a clean error state
    if (resolve_fixed_scratch(c)) return bail(PIC_E_DEVICE);
    // ---- per case ----
    size_t hist_total = 0;
    for (int k = 0; k < n_cases; ++k) {
        const pic_case_config& g = cases[k];
        HostCase& h = c->hc[k];
        Case& C = c->cases_h[k];
        std::memset(&C, 0, sizeof(Case));
        h.cfg = g;
        h.cfg.cell_dx_m = nullptr;   // the caller's array is copied
        if (g.cell_dx_m) h.cell_w.assign(g.cell_dx_m, g.cell_dx_m + g.n_cells);
        const int N = g.n_cells;
        const double dx = g.gap_m / N, dt = g.dt_s;
        h.vscale = dt / dx;
        C.n_cells = N;
        C.bc = g.bc;
        C.scheme = g.scheme;
        C.gather = g.gather;
        C.collisions = g.collisions;
        C.history_len = g.history_steps;
        C.nonuniform = g.cell_dx_m ? 1 : 0;
        C.ion_sub = g.ion_subcycle > 1 ? g.ion_subcycle : 1;
        C.dx = dx;
        C.dt = dt;
        C.rf_volts = g.rf_volts;
        C.rf_omega = 6.283185307179586476925286766559 * g.rf_freq_hz;
        C.rf_freq = g.rf_freq_hz;
        C.background_rho = g.background_rho;
        C.key0 = (uint32_t)g.seed;
        C.key1 = (uint32_t)(g.seed >> 32);
        c->maxN = std::max(c->maxN, N);
        c->any_dual = c->any_dual || dual_chi(g.scheme, g.gather);
        c->dep_lds_max = std::max(c->dep_lds_max, deposit_lds(N, dual_chi(g.scheme, g.gather),
                                                              g.cell_dx_m != nullptr));
        // Eq. (1): omega_p dt < 2 for the explicit leap-frog
        if (g.scheme == PIC_EXPLICIT && !(flags & PIC_FLAG_ALLOW_UNSTABLE)) {
            const pic_species_init& e = species[2 * k];
            std::vector<int64_t> cnt(N, 0);
            std::vector<int32_t> cells(e.n);
            if (e.n > 0 && hipMemcpy(cells.data(), e.cell, sizeof(int32_t) * e.n,
                                     hipMemcpyDefault) != hipSuccess)
                return bail(fail(c, PIC_E_DEVICE, "copy cells"));
            for (int32_t cc : cells)
                if (cc >= 0 && cc < N) cnt[cc]++;
            int64_t mx = cnt.empty() ? 0 : *std::max_element(cnt.begin(), cnt.end());
            double ne = mx * e.weight / dx;
            double wp = std::sqrt(ne * e.q_C * e.q_C / (EPS0 * e.m_kg));
            if (wp * dt >= 2.0) {
                c->err = "explicit case violates omega_p dt < 2";
                destroy_ctx(c);
                return PIC_E_UNSTABLE;
            }
        }
        for (int s = 0; s < 2; ++s) {
            const pic_species_init& sp = species[2 * k + s];
            Species& S = C.sp[s];
            h.q[s] = sp.q_C;
            h.m[s] = sp.m_kg;
            h.w[s] = sp.weight;
            h.cap[s] = std::max<int64_t>(sp.capacity, 1);
            h.n0[s] = sp.n;
            S.capacity = h.cap[s];
            const double m = sp.m_kg, q = sp.q_C, w = sp.weight;
            S.accel = q / m * dt * dt / dx;
            S.qw_dx = q * w / dx;
            S.kin_unit = 0.5 * m * w * (dx / dt) * (dx / dt);
            // subcycled ions respond over their own step K dt
            const double hs = (s == 1 && g.ion_subcycle > 1) ? (double)g.ion_subcycle : 1.0;
            S.chi_coef = 0.5 * dt * dt * hs * hs * q * q * w / (m * EPS0 * dx);
            S.dens_unit = w / dx;
            const double eps_unit = 0.5 * m * (dx / dt) * (dx / dt) / QE;
            S.eps_unit = (float)eps_unit;
            S.opal_B = (float)g.opal_B_eV;
            S.recoil2 = (float)(2.0 * species[2 * k].m_kg / (g.gas_mass_kg > 0 ? g.gas_mass_kg : 1.0));
            S.vth_neutral = (float)(std::sqrt(KB * g.gas_temp_K / (g.gas_mass_kg > 0 ? g.gas_mass_kg : 1.0)) * dt / dx);
            S.vth_newion = (float)(std::sqrt(KB * g.gas_temp_K / species[2 * k + 1].m_kg) * dt / dx);
            S.eedf_scale = 2.0f;   // 0.5 eV bins
            double* c64 = h.c64[s];
            c64[0] = eps_unit;
            c64[1] = g.opal_B_eV;
            c64[2] = 2.0 * species[2 * k].m_kg / (g.gas_mass_kg > 0 ? g.gas_mass_kg : 1.0);
            c64[3] = std::sqrt(KB * g.gas_temp_K / (g.gas_mass_kg > 0 ? g.gas_mass_kg : 1.0)) * dt / dx;
            c64[4] = std::sqrt(KB * g.gas_temp_K / species[2 * k + 1].m_kg) * dt / dx;
            for (int p = 5; p < 12; ++p) c64[p] = p >= 8 ? -1.0 : 0.0;
            for (int p = 0; p < kMaxProc; ++p) {
                S.kind[p] = -1;
                S.thr_v2[p] = -1.0f;
            }
            S.n_proc = g.collisions ? (int32_t)proc[s].size() : 0;
            // per-case collision table: sigma * n_g (dx/dt) / nu_max
            if (S.n_proc > 0) {
                const pic_xsec* a = proc[s][0];
                const double numax = nu_max(proc[s], g.gas_density_m3, m);
                // a subcycled species takes its trials with the step K dt
                const double pnull = 1.0 - std::exp(-numax * dt * (s == 1 ? C.ion_sub : 1));
                S.cand_thr = numax > 0 ? candidate_threshold(pnull) : 0u;
                S.inv_log1mp = (pnull > 0.0 && pnull < 1.0) ? 1.0 / std::log1p(-pnull) : 0.0;
                const double scale = numax > 0 ? g.gas_density_m3 * (dx / dt) / numax : 0.0;
                h.scale[s] = scale;
                h.pnull[s] = pnull;
                S.t_scale = (float)(eps_unit / a->de_eV);
                S.t_off = (float)(-a->e0_eV / a->de_eV);
                S.t_max = (float)(a->n - 1);
                c64[5] = eps_unit / a->de_eV;
                c64[6] = -a->e0_eV / a->de_eV;
                c64[7] = (double)(a->n - 1);
                for (int p = 0; p < S.n_proc; ++p) {
                    S.kind[p] = proc[s][p]->kind;
                    S.thr_v2[p] = proc[s][p]->threshold_eV > 0
                                      ? (float)(proc[s][p]->threshold_eV / eps_unit)
                                      : -1.0f;
                    c64[8 + p] = proc[s][p]->threshold_eV > 0 ? proc[s][p]->threshold_eV / eps_unit
                                                              : -1.0;
                }
                if (s == 0) {
                    std::vector<float> t(4 * (size_t)a->n, 0.0f);
                    for (int32_t i = 0; i < a->n; ++i)
                        for (int p = 0; p < S.n_proc; ++p)
                            t[4 * i + p] = (float)(proc[s][p]->sigma_m2[i] * scale);
                    float4* d = nullptr;
                    if (dalloc(c, h.allocs, &d, (size_t)a->n)) return bail(PIC_E_NOMEM);
                    INITCHK(hipMemcpy(d, t.data(), t.size() * 4, hipMemcpyHostToDevice));
                    S.tab_e = d;
                    // Bound table: for the intervals k in [b K, (b+1) K) the
                    // cumulative sum the kernel compares u1 with is at most
                    // sum_p max sigma_p over the points b K .. (b+1) K times the
                    // largest speed of the bin (a 1e-5 margin covers float
                    // rounding); u1 above it is a null collision for certain.
                    const int K = std::max(1, (a->n - 1 + kBoundBins - 1) / kBoundBins);
                    std::vector<float> bnd(kBoundBins, 0.0f);
                    for (int b = 0; b < kBoundBins; ++b) {
                        const int k_lo = b * K;
                        if (k_lo > a->n - 1) {
                            bnd[b] = bnd[b > 0 ? b - 1 : 0];
                            continue;
                        }
                        const int k_hi = std::min((b + 1) * K, a->n - 1);
                        double sum = 0.0;
                        for (int p = 0; p < S.n_proc; ++p) {
                            float mx = 0.0f;
                            for (int k2 = k_lo; k2 <= k_hi; ++k2) mx = std::max(mx, t[4 * k2 + p]);
                            sum += mx;
                        }
                        const double t_hi = (double)k_hi + 1.0;   // slack of one interval
                        const double v2 = std::max(0.0, (t_hi - c64[6]) / c64[5]);
                        bnd[b] = (float)(sum * std::sqrt(v2) * (1.0 + 1e-5));
                    }
                    float* db = nullptr;
                    if (dalloc(c, h.allocs, &db, (size_t)kBoundBins)) return bail(PIC_E_NOMEM);
                    INITCHK(hipMemcpy(db, bnd.data(), 4 * (size_t)kBoundBins, hipMemcpyHostToDevice));
                    S.cbound = db;
                    S.bound_k = K;
                } else {
                    std::vector<float> t((size_t)a->n);
                    for (int32_t i = 0; i < a->n; ++i) t[i] = (float)(proc[s][0]->sigma_m2[i] * scale);
                    float* d = nullptr;
                    if (dalloc(c, h.allocs, &d, (size_t)a->n)) return bail(PIC_E_NOMEM);
                    INITCHK(hipMemcpy(d, t.data(), t.size() * 4, hipMemcpyHostToDevice));
                    S.tab_i = d;
                }
            }
            // particle store (two copies)
            const size_t cap = (size_t)h.cap[s];
            int rc = 0;
            rc |= dalloc(c, h.allocs, &S.cell, cap);
            rc |= dalloc(c, h.allocs, &S.off, cap);
            rc |= dalloc(c, h.allocs, &S.vx, cap);
            rc |= dalloc(c, h.allocs, &S.rec, cap);
            rc |= dalloc(c, h.allocs, &S.abar, cap);
            rc |= dalloc(c, h.allocs, &S.cell2, cap);
            rc |= dalloc(c, h.allocs, &S.off2, cap);
            rc |= dalloc(c, h.allocs, &S.vx2, cap);
            rc |= dalloc(c, h.allocs, &S.rec2, cap);
            rc |= dalloc(c, h.allocs, &S.abar2, cap);
            rc |= dalloc(c, h.allocs, &S.cq_idx, cap);
            rc |= dalloc(c, h.allocs, &S.cq_vn, cap);
            rc |= dalloc(c, h.allocs, &S.cq_ab, cap);
            rc |= dalloc(c, h.allocs, &S.cq_w, cap);
            rc |= dalloc(c, h.allocs, &S.cq_o, cap);
            if (rc) return bail(PIC_E_NOMEM);
            if (sp.n > 0) {
                const size_t n = (size_t)sp.n;
                INITCHK(hipMemcpy(S.cell, sp.cell, 4 * n, hipMemcpyDefault));
                INITCHK(hipMemcpy(S.off, sp.off, 4 * n, hipMemcpyDefault));
                INITCHK(hipMemcpy(S.vx, sp.vx, 4 * n, hipMemcpyDefault));
                {
                    // id, vy, vz into the 16-byte records
                    std::vector<float> yy(n), zz(n);
                    std::vector<uint64_t> ii(n);
                    INITCHK(hipMemcpy(yy.data(), sp.vy, 4 * n, hipMemcpyDefault));
                    INITCHK(hipMemcpy(zz.data(), sp.vz, 4 * n, hipMemcpyDefault));
                    INITCHK(hipMemcpy(ii.data(), sp.id, 8 * n, hipMemcpyDefault));
                    std::vector<uint32_t> rr(4 * n);
                    for (size_t i = 0; i < n; ++i) {
                        rr[4 * i] = (uint32_t)ii[i];
                        rr[4 * i + 1] = (uint32_t)(ii[i] >> 32);
                        std::memcpy(&rr[4 * i + 2], &yy[i], 4);
                        std::memcpy(&rr[4 * i + 3], &zz[i], 4);
                    }
                    INITCHK(hipMemcpy(S.rec, rr.data(), 16 * n, hipMemcpyHostToDevice));
                }
                if (sp.abar) INITCHK(hipMemcpy(S.abar, sp.abar, 4 * n, hipMemcpyDefault));
                // positions must lie inside the gap / box
                std::vector<int32_t> cc(n);
                std::vector<float> oo(n);
                INITCHK(hipMemcpy(cc.data(), S.cell, 4 * n, hipMemcpyDeviceToHost));
                INITCHK(hipMemcpy(oo.data(), S.off, 4 * n, hipMemcpyDeviceToHost));
                for (size_t i = 0; i < n; ++i)
                    if (cc[i] < 0 || cc[i] >= N || !(oo[i] >= 0.0f) || !(oo[i] < 1.0f)) {
                        fprintf(stderr, "pic_init: case %d species %d particle %zu out of range\n",
                                k, s, i);
                        return bail(PIC_E_INVAL);
                    }
                // the device cell word carries the null-collision waiting time
                if (sp.mcc_wait) {
                    std::vector<uint32_t> ww(n);
                    INITCHK(hipMemcpy(ww.data(), sp.mcc_wait, 4 * n, hipMemcpyDefault));
                    for (size_t i = 0; i < n; ++i) {
                        if (ww[i] > (PIC_WAIT_MAX | PIC_WAIT_CAPPED)) {
                            fprintf(stderr, "pic_init: case %d species %d particle %zu: bad wait\n",
                                    k, s, i);
                            return bail(PIC_E_INVAL);
                        }
                        // count at the species' first move -> expiry field
                        const int ks = s == 1 ? std::max(1, (int)g.ion_subcycle) : 1;
                        const uint32_t clk = clock_from(g.start_step, ks, S.n_proc > 0);
                        cc[i] |= (int32_t)(wait_field(clk, ww[i]) << kCellWordBits);
                    }
                    INITCHK(hipMemcpy(S.cell, cc.data(), 4 * n, hipMemcpyHostToDevice));
                }
            }
        }
        // grids
        int rc = 0;
        for (int s = 0; s < 2; ++s) {
            rc |= dalloc(c, h.allocs, &C.dep_cnt[s], N + 1);   // node N: quadratic deposit
            rc |= dalloc(c, h.allocs, &C.dep_w[s], N + 1);
            if (dual_chi(C.scheme, C.gather)) {
                rc |= dalloc(c, h.allocs, &C.chi_cnt[s], N + 1);
                rc |= dalloc(c, h.allocs, &C.chi_w[s], N + 1);
                if (C.nonuniform) {
                    rc |= dalloc(c, h.allocs, &C.chl_w0[s], N + 1);
                    rc |= dalloc(c, h.allocs, &C.chl_w2[s], N + 1);
                }
            }
            rc |= dalloc(c, h.allocs, &C.ehat[s], N);
            rc |= dalloc(c, h.allocs, &C.qfix[s], N + 1);
            rc |= dalloc(c, h.allocs, &C.ccount[s], N);
            rc |= dalloc(c, h.allocs, &C.dens_acc[s], N + 1);
            rc |= dalloc(c, h.allocs, &C.heat_acc[s], N);
        }
        rc |= dalloc(c, h.allocs, &C.E, N);
        rc |= dalloc(c, h.allocs, &C.phi, N + 1);
        rc |= dalloc(c, h.allocs, &C.rho, N + 1);
        rc |= dalloc(c, h.allocs, &C.chi, N);
        rc |= dalloc(c, h.allocs, &C.eedf_acc, kEedfBins);
        pic_ledger* hist = nullptr;
        rc |= dalloc(c, h.allocs, &hist, (size_t)g.history_steps + 1);
        C.history = hist;
        if (!h.cell_w.empty()) {
            // the moves take r_c = dx / w_c (float), the solve w_c / dx (double)
            rc |= dalloc(c, h.allocs, &C.cell_r, N);
            rc |= dalloc(c, h.allocs, &C.cell_wr, N);
            rc |= dalloc(c, h.allocs, &C.cell_run, N);
        }
        if (rc) return bail(PIC_E_NOMEM);
        if (!h.cell_w.empty()) {
            std::vector<float> r(N);
            std::vector<double> wr(N);
            for (int j = 0; j < N; ++j) {
                r[j] = (float)(C.dx / h.cell_w[j]);
                wr[j] = h.cell_w[j] / C.dx;
            }
            // runs of equal ratios: first | last << 16
            std::vector<uint32_t> run(N);
            for (int j = 0, a = 0; j < N; ++j) {
                if (j + 1 == N || r[j + 1] != r[j]) {
                    for (int t = a; t <= j; ++t) run[t] = (uint32_t)a | ((uint32_t)j << 16);
                    a = j + 1;
                }
            }
            INITCHK(hipMemcpy(C.cell_r, r.data(), 4 * (size_t)N, hipMemcpyHostToDevice));
            INITCHK(hipMemcpy(C.cell_wr, wr.data(), 8 * (size_t)N, hipMemcpyHostToDevice));
            INITCHK(hipMemcpy(C.cell_run, run.data(), 4 * (size_t)N, hipMemcpyHostToDevice));
        }
        h.hist_off[0] = hist_total;
        h.hist_off[1] = hist_total + N;
        hist_total += 2 * (size_t)N;
    }
    size_t lds_need = fin_lds(c->maxN);
    for (int k = 0; k < n_cases; ++k)
        lds_need = std::max(lds_need, case_lds(cases[k].n_cells,
                                               dual_chi(cases[k].scheme, cases[k].gather),
                                               cases[k].cell_dx_m != nullptr));
    if (set_lds_limits(c, lds_need))
        return bail(PIC_E_INVAL);
    // ---- context arrays ----
    c->hist_total = hist_total;
    if (dalloc(c, c->allocs, &c->d_cases, n_cases) || dalloc(c, c->allocs, &c->d_state, n_cases) ||
        dalloc(c, c->allocs, &c->d_hist, hist_total) ||
        dalloc(c, c->allocs, &c->d_cursor, hist_total) ||
        dalloc(c, c->allocs, &c->d_hist_off, 2 * (size_t)n_cases))
        return bail(PIC_E_NOMEM);
    {
        std::vector<int64_t> ho(2 * n_cases);
        for (int k = 0; k < n_cases; ++k) {
            ho[2 * k] = (int64_t)c->hc[k].hist_off[0];
            ho[2 * k + 1] = (int64_t)c->hc[k].hist_off[1];
        }
        INITCHK(hipMemcpy(c->d_hist_off, ho.data(), 8 * ho.size(), hipMemcpyHostToDevice));
    }
    build_work(c);
    if (upload_work(c)) return bail(PIC_E_DEVICE);
    INITCHK(hipMemcpy(c->d_cases, c->cases_h.data(), sizeof(Case) * n_cases,
                        hipMemcpyHostToDevice));
    {
        std::vector<State> st(n_cases);
        std::memset(st.data(), 0, sizeof(State) * n_cases);
        for (int k = 0; k < n_cases; ++k) {
            st[k].step = cases[k].start_step;
            st[k].ledger_step = cases[k].start_step;
            for (int s = 0; s < 2; ++s) {
                st[k].n_slots[s] = (int32_t)species[2 * k + s].n;
                st[k].n_live[s] = (int32_t)species[2 * k + s].n;
            }
        }
        INITCHK(hipMemcpy(c->d_state, st.data(), sizeof(State) * n_cases,
                            hipMemcpyHostToDevice));
    }
    // ---- set-up on the device: units, D1 start-up, sort, deposit, solve ----
    {
        // mode bits: 1 unit conversion, 2 D1 start-up (both only for inputs in
        // physical units; an internal-units state is already predicted), 8 << s
        // draw the waits of species s (loaded without them)
        const int base_mode = (flags & PIC_FLAG_INTERNAL_UNITS) ? 0 : 3;
        // one kernel per case scale: vscale differs per case, so pass per launch
        for (int k = 0; k < n_cases; ++k) {
            int mode = base_mode;
            for (int s = 0; s < 2; ++s)
                if (!species[2 * k + s].mcc_wait) mode |= 8 << s;
            // restrict the launch to this case's workgroups
            Params p = params(c, mode);
            p.work = c->d_work + c->cases_h[k].first_block;
            hipLaunchKernelGGL(k_init_species, dim3(c->cases_h[k].n_blocks), dim3(kBlock), 0,
                               c->stream, p, c->hc[k].vscale, c->hc[k].vscale);
        }
        INITCHK(hipGetLastError());
        if (compaction(c)) return bail(PIC_E_DEVICE);
        Params p = params(c, 0);
        hipLaunchKernelGGL(k_deposit, dim3(c->n_blocks), dim3(kBlock),
                           c->dep_lds_max, c->stream, p);
        hipLaunchKernelGGL(k_solve, dim3(n_cases), dim3(kFinBlock), fin_lds(c->maxN),
                           c->stream, p);
        INITCHK(hipGetLastError());
        INITCHK(hipStreamSynchronize(c->stream));
    }
    *out = c;
    return PIC_OK;
}

namespace {

void destroy_ctx(pic_ctx* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    pic__fp64_free(c);
    for (auto& h : c->hc)
        for (void* p : h.allocs) (void)hipFree(p);
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->d_work) (void)hipFree(c->d_work);
    if (c->d_pd) (void)hipFree(c->d_pd);
    if (c->d_pu) (void)hipFree(c->d_pu);
    if (c->d_cand_n) (void)hipFree(c->d_cand_n);
    if (c->d_cwork) (void)hipFree(c->d_cwork);
    drop_graph(c);
    for (hipEvent_t e : c->ev.ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->graph.ev.ev) (void)hipEventDestroy(e);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->stream2) (void)hipStreamDestroy(c->stream2);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int check_flags(pic_ctx* c)
{
    std::vector<State> st(c->n_cases);
    HIPCHK(c, hipMemcpy(st.data(), c->d_state, sizeof(State) * c->n_cases, hipMemcpyDeviceToHost));
    int rc = PIC_OK;
    for (int k = 0; k < c->n_cases; ++k) {
        if (st[k].flags & 1) return fail(c, PIC_E_DIVERGED, "non-finite field or energy");
        if (st[k].flags & 2) rc = fail(c, PIC_E_CAPACITY, "particle capacity exceeded");
    }
    return rc;
}

// Longest sort period captured into one graph (a graph holds 3-5 nodes per step).
constexpr int kMaxGraphPeriod = 1024;

// Make sure the pool holds at least `pairs` event pairs.
int reserve_events(pic_ctx* c, EventPool& pool, int pairs)
{
    while ((int)pool.ev.size() < 2 * pairs) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        pool.ev.push_back(e);
    }
    return PIC_OK;
}

// The launches of one step on the context's stream: per scheme group the
// particle pass and the collision kernel, then the finalizer of every case;
// the compaction follows when the sort period ends.  With `pool`, HIP events
// bracket the particle and collision kernels (as event nodes under capture).
// A batch with both schemes runs the implicit group, with the finalizer of
// its cases, on the second stream (not while events bracket the kernels,
// under capture or in the call that allocates nothing), so that the two
// groups overlap and need no join in every step.
int join_streams(pic_ctx* c)
{
    if (!c->forked) return PIC_OK;
    HIPCHK(c, hipEventRecord(c->ev_join, c->stream2));
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
    c->forked = false;
    return PIC_OK;
}

using FinKernel = void (*)(Params, int);
FinKernel fin_kernel(bool dual, bool plain)
{
    return dual ? k_finalize<true, false> : plain ? k_finalize<false, true> : k_finalize<false, false>;
}

int enqueue_step(pic_ctx* c, bool diag, EventPool* pool, bool capturing)
{
    auto record = [&](hipEvent_t e) {
        return capturing ? hipEventRecordWithFlags(e, c->stream, hipEventRecordExternal)
                         : hipEventRecord(e, c->stream);
    };
    const bool split = c->grp_cnt[0] && c->grp_cnt[1] && !pool && !capturing && !c->use_fixed;
    if (!split && join_streams(c)) return PIC_E_DEVICE;
    if (split && !c->forked) {
        HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
        HIPCHK(c, hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
        c->forked = true;
    }
    for (int gi = 0; gi < 2; ++gi) {
        // the implicit group first, so that it starts on its stream first
        const int g = split ? 1 - gi : gi;
        if (!c->grp_cnt[g]) continue;
        hipStream_t sg = split && g == 1 ? c->stream2 : c->stream;
        Params p = params(c, c->grp_off[g]);
        Params pc = params(c, c->cgrp_off[g]);
        auto ks = step_kernel(g, diag, c->grp_gt[g], c->grp_dual[g], c->grp_plain[g]);
        auto kc = collide_kernel(g, diag, c->grp_dual[g], c->grp_plain[g]);
        for (int kind = 0; kind < 2; ++kind) {
            if (kind == 1 && !c->cgrp_cnt[g]) continue;
            const bool rec = pool && pool->used + 2 <= (int)pool->ev.size();
            if (rec) HIPCHK(c, record(pool->ev[pool->used]));
            if (kind == 0)
                hipLaunchKernelGGL(ks, dim3(c->grp_cnt[g]), dim3(kBlock),
                                   c->grp_slds[g][diag ? 1 : 0], sg, p);
            else
                hipLaunchKernelGGL(kc, dim3(c->cgrp_cnt[g]), dim3(kBlock),
                                   c->grp_clds[g], sg, pc);
            if (rec) {
                HIPCHK(c, record(pool->ev[pool->used + 1]));
                pool->used += 2;
                pool->kind.push_back(kind);
            }
        }
        // split: the finalizer of the group's cases (the workgroups of the
        // other group's cases return at once)
        if (split)
            hipLaunchKernelGGL(fin_kernel(c->grp_dual[g], c->grp_plain[g]), dim3(2 * c->n_cases),
                               dim3(kFinStep), fin_lds(c->maxN), sg, params(c, g), diag ? 1 : 0);
    }
    if (!split)
        hipLaunchKernelGGL(fin_kernel(c->any_dual, c->grp_plain[0] && c->grp_plain[1]),
                           dim3(2 * c->n_cases), dim3(kFinStep), fin_lds(c->maxN), c->stream,
                           params(c, -1), diag ? 1 : 0);
    HIPCHK(c, hipGetLastError());
    if (++c->since_sort >= c->sort_every) {
        if (join_streams(c)) return PIC_E_DEVICE;
        if (compaction(c)) return PIC_E_DEVICE;
    }
    return PIC_OK;
}

bool timed_step(const pic_ctx* c, int64_t step)
{
    return c->timing_every > 0 && step % c->timing_every == 0;
}

void drop_graph(pic_ctx* c)
{
    if (c->graph.exec) {
        if (c->stream) (void)hipStreamSynchronize(c->stream);
        (void)hipGraphExecDestroy(c->graph.exec);
    }
    c->graph.exec = nullptr;
    c->graph.period = 0;
}

// Capture one sort period, starting at a period boundary, into c->graph.
int capture_period(pic_ctx* c)
{
    drop_graph(c);
    int timed = 0;
    for (int j = 0; j < c->sort_every; ++j) timed += timed_step(c, j) ? 1 : 0;
    if (reserve_events(c, c->graph.ev, 4 * timed)) return PIC_E_DEVICE;
    c->graph.ev.used = 0;
    c->graph.ev.kind.clear();
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = PIC_OK;
    const int64_t since0 = c->since_sort;
    for (int j = 0; j < c->sort_every && rc == PIC_OK; ++j)
        rc = enqueue_step(c, false, timed_step(c, j) ? &c->graph.ev : nullptr, true);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &graph);
    c->since_sort = since0;
    if (rc != PIC_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(c, PIC_E_DEVICE, std::string("hipStreamEndCapture: ") +
                                             hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(&c->graph.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        c->graph.exec = nullptr;
        return fail(c, PIC_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    c->graph.period = c->sort_every;
    return PIC_OK;
}

// Sum the elapsed times of the pool's event pairs by kernel kind.
void add_times(const EventPool& pool, double ms[2], int64_t launches[2])
{
    for (int e = 0; e + 1 < pool.used; e += 2) {
        float t = 0.0f;
        const int kind = pool.kind[e / 2];
        if (hipEventElapsedTime(&t, pool.ev[e], pool.ev[e + 1]) == hipSuccess) {
            ms[kind] += t;
            launches[kind]++;
        }
    }
}

// Advance n steps.  With `bracket`, events bracket the whole enqueued
// sequence on the stream (used to time autotuning trials).
int run_steps(pic_ctx* c, int64_t n, int which, hipEvent_t* bracket = nullptr)
{
    if (c->failed) return fail(c, PIC_E_STATE, "context failed earlier: " + c->err);
    if (n < 0) return fail(c, PIC_E_INVAL, "negative step count");
    for (int k = 0; k < c->n_cases; ++k)
        if (which >= 0 && c->hc[k].cfg.scheme != which)
            return fail(c, PIC_E_INVAL, "a case of the context uses the other scheme");
    const bool graphs = c->use_graph && c->diag_every == 0 && c->sort_every <= kMaxGraphPeriod;
    // host-launched steps: at most one partial period at each end when graphs are used
    int64_t host_steps = graphs ? std::min<int64_t>(n, 2 * (int64_t)c->sort_every) : n;
    int64_t timed = 0;
    if (c->timing_every > 0) timed = host_steps / c->timing_every + 1;
    // up to two timed kernels per scheme group and step
    if (reserve_events(c, c->ev, (int)std::min<int64_t>(4 * timed, 1 << 20))) return PIC_E_DEVICE;
    c->ev.used = 0;
    c->ev.kind.clear();
    int64_t replays = 0;
    if (bracket) HIPCHK(c, hipEventRecord(bracket[0], c->stream));
    for (int64_t it = 0; it < n;) {
        if (graphs && c->since_sort == 0 && n - it >= c->sort_every) {
            if (join_streams(c)) return PIC_E_DEVICE;
            if (c->graph.period != c->sort_every || !c->graph.exec)
                if (capture_period(c)) return PIC_E_DEVICE;
            HIPCHK(c, hipGraphLaunch(c->graph.exec, c->stream));
            c->steps_taken += c->sort_every;
            it += c->sort_every;
            ++replays;
            continue;
        }
        const bool diag = c->diag_every > 0 && (c->steps_taken % c->diag_every == 0);
        // the step index within the period decides timing, as in a captured period
        if (enqueue_step(c, diag, timed_step(c, c->since_sort) ? &c->ev : nullptr, false))
            return PIC_E_DEVICE;
        c->steps_taken++;
        ++it;
    }
    if (join_streams(c)) return PIC_E_DEVICE;
    if (bracket) HIPCHK(c, hipEventRecord(bracket[1], c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double ms[2] = {0.0, 0.0};
    int64_t launches[2] = {0, 0};
    add_times(c->ev, ms, launches);
    if (replays > 0) add_times(c->graph.ev, ms, launches);
    c->last_ms = ms[0];
    c->last_launches = launches[0];
    c->last_ms_coll = ms[1];
    c->last_launches_coll = launches[1];
    return check_flags(c);
}

}  // namespace

extern "C" int pic_step_explicit(pic_ctx* ctx, int64_t n)
{
    if (!ctx) return PIC_E_INVAL;
    return run_steps(ctx, n, PIC_EXPLICIT);
}

extern "C" int pic_step_implicit(pic_ctx* ctx, int64_t n)
{
    if (!ctx) return PIC_E_INVAL;
    return run_steps(ctx, n, PIC_IMPLICIT_D1);
}

extern "C" int pic_step(pic_ctx* ctx, int64_t n)
{
    if (!ctx) return PIC_E_INVAL;
    return run_steps(ctx, n, -1);
}

extern "C" int pic_step_noalloc(pic_ctx* ctx, int64_t n)
{
    if (!ctx) return PIC_E_INVAL;
    if (ctx->failed) return fail(ctx, PIC_E_STATE, "context failed earlier: " + ctx->err);
    if (n < 0) return fail(ctx, PIC_E_INVAL, "negative step count");
    if (!ctx->fixed_scratch) return fail(ctx, PIC_E_STATE, "no fixed scratch on this device");
    int dev = -1;
    HIPCHK(ctx, hipGetDevice(&dev));
    if (dev != ctx->device) return fail(ctx, PIC_E_INVAL, "the context's device is not current");
    // layout of the step's scratch in the fixed array (256-byte aligned parts)
    const size_t rows = ctx->work.size();
    size_t used = 0;
    auto take = [&](size_t bytes) {
        const size_t at = used;
        used += (bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t o_pd = take(sizeof(double) * PD_N * rows);
    const size_t o_pu = take(sizeof(unsigned) * PU_N * rows);
    const size_t o_cn = take(sizeof(int32_t) * rows);
    const size_t o_hist = take(sizeof(uint32_t) * ctx->hist_total);
    const size_t o_cur = take(sizeof(uint32_t) * ctx->hist_total);
    if (used > kFixedScratchBytes)
        return fail(ctx, PIC_E_INVAL,
                    "pic_step_noalloc: the schedule needs " + std::to_string(used) +
                        " bytes of scratch (" + std::to_string(rows) +
                        " workgroups), the fixed array holds " +
                        std::to_string(kFixedScratchBytes) + " (use a larger tile)");
    char* base = (char*)ctx->fixed_scratch;
    ctx->fx_pd = (double*)(base + o_pd);
    ctx->fx_pu = (unsigned*)(base + o_pu);
    ctx->fx_cand_n = (int32_t*)(base + o_cn);
    ctx->fx_hist = (uint32_t*)(base + o_hist);
    ctx->fx_cursor = (uint32_t*)(base + o_cur);
    // the histograms must start at zero (every compaction leaves them zero;
    // an earlier call may have left anything); the partial rows and counts
    // are written whole by each step's particle pass before they are read
    if (ctx->hist_total > 0) {
        const uint32_t nh = (uint32_t)ctx->hist_total;
        hipLaunchKernelGGL(k_fill_u32, dim3(std::min<uint32_t>((nh + 255) / 256, 1024)),
                           dim3(256), 0, ctx->stream, ctx->fx_hist, nh, 0u);
    }
    ctx->use_fixed = true;
    int rc = PIC_OK;
    for (int64_t it = 0; it < n && rc == PIC_OK; ++it) {
        const bool diag = ctx->diag_every > 0 && (ctx->steps_taken % ctx->diag_every == 0);
        rc = enqueue_step(ctx, diag, nullptr, false);
        if (rc == PIC_OK) ctx->steps_taken++;
    }
    ctx->use_fixed = false;
    if (rc != PIC_OK) return rc;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->last_ms = ctx->last_ms_coll = 0.0;
    ctx->last_launches = ctx->last_launches_coll = 0;
    // the flags of every case, read without host containers
    int out = PIC_OK;
    for (int k = 0; k < ctx->n_cases; ++k) {
        State st;
        HIPCHK(ctx, hipMemcpy(&st, ctx->d_state + k, sizeof(State), hipMemcpyDeviceToHost));
        if (st.flags & 1) return fail(ctx, PIC_E_DIVERGED, "non-finite field or energy");
        if (st.flags & 2) out = fail(ctx, PIC_E_CAPACITY, "particle capacity exceeded");
    }
    return out;
}

extern "C" int pic_last_timing(const pic_ctx* ctx, double* ms, int64_t* launches)
{
    if (!ctx) return PIC_E_INVAL;
    if (ms) *ms = ctx->last_ms;
    if (launches) *launches = ctx->last_launches;
    return PIC_OK;
}

extern "C" int pic_last_timing_collide(const pic_ctx* ctx, double* ms, int64_t* launches)
{
    if (!ctx) return PIC_E_INVAL;
    if (ms) *ms = ctx->last_ms_coll;
    if (launches) *launches = ctx->last_launches_coll;
    return PIC_OK;
}

extern "C" int pic_set_schedule(pic_ctx* ctx, int32_t sort_every, int32_t diag_every, int32_t tile)
{
    if (!ctx) return PIC_E_INVAL;
    if (ctx->failed) return fail(ctx, PIC_E_STATE, ctx->err);
    if (sort_every < 1 || diag_every < 0 || tile < 0 || (tile > 0 && (tile % kBlock || tile > kMaxTile + 1)))
        return fail(ctx, PIC_E_INVAL, "bad schedule");
    drop_graph(ctx);   // the captured period holds the old schedule's launches
    ctx->sort_every = sort_every;
    ctx->diag_every = diag_every;
    if (tile > 0 && tile != ctx->tile) {
        // the device case table holds the current buffer pointers: read it back
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        HIPCHK(ctx, hipMemcpy(ctx->cases_h.data(), ctx->d_cases, sizeof(Case) * ctx->n_cases,
                              hipMemcpyDeviceToHost));
        ctx->tile = std::min(tile, kMaxTile);
        build_work(ctx);
        if (upload_work(ctx)) return PIC_E_DEVICE;
        HIPCHK(ctx, hipMemcpy(ctx->d_cases, ctx->cases_h.data(), sizeof(Case) * ctx->n_cases,
                              hipMemcpyHostToDevice));
    }
    return PIC_OK;
}

extern "C" int pic_set_launch(pic_ctx* ctx, int32_t graph, int32_t timing_every)
{
    if (!ctx) return PIC_E_INVAL;
    if (ctx->failed) return fail(ctx, PIC_E_STATE, ctx->err);
    if ((graph != 0 && graph != 1) || timing_every < 0)
        return fail(ctx, PIC_E_INVAL, "bad launch mode");
    if (graph && !ctx->stream)
        return fail(ctx, PIC_E_INVAL, "graph replay needs a stream other than the null stream");
    drop_graph(ctx);
    ctx->use_graph = graph == 1;
    ctx->timing_every = timing_every;
    return PIC_OK;
}

extern "C" int pic_set_store_policy(pic_ctx* ctx, int32_t nontemporal)
{
    if (!ctx) return PIC_E_INVAL;
    if (ctx->failed) return fail(ctx, PIC_E_STATE, ctx->err);
    if (nontemporal != 0 && nontemporal != 1) return fail(ctx, PIC_E_INVAL, "bad store policy");
    if (ctx->nt_store != (nontemporal == 1)) drop_graph(ctx);   // captured launches hold the old one
    ctx->nt_store = nontemporal == 1;
    return PIC_OK;
}

namespace {

// Device milliseconds per step of `steps` real steps at the current schedule,
// after `warm` untimed steps.
int timed_trial(pic_ctx* c, int warm, int64_t steps, hipEvent_t* ev, double* ms_per_step)
{
    if (warm > 0) {
        const int r = run_steps(c, warm, -1);
        if (r) return r;
    }
    const int rc = run_steps(c, steps, -1, ev);
    if (rc) return rc;
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, ev[0], ev[1]));
    *ms_per_step = (double)ms / (double)steps;
    return PIC_OK;
}

}  // namespace

extern "C" int pic_autotune(pic_ctx* ctx, const int32_t* tiles, int32_t n_tiles,
                            const int32_t* sorts, int32_t n_sorts, int32_t steps_per_trial,
                            int32_t* tile_out, int32_t* sort_out, double* ms_out)
{
    if (!ctx) return PIC_E_INVAL;
    if (ctx->failed) return fail(ctx, PIC_E_STATE, ctx->err);
    static const int32_t kTiles[] = {1024, 2048, 4096, 8192, 16384, 32512};
    static const int32_t kSorts[] = {16, 32, 64, 128};
    if (!tiles) {
        tiles = kTiles;
        n_tiles = (int32_t)(sizeof(kTiles) / sizeof(kTiles[0]));
    }
    if (!sorts) {
        sorts = kSorts;
        n_sorts = (int32_t)(sizeof(kSorts) / sizeof(kSorts[0]));
    }
    if (n_tiles < 1 || n_sorts < 1 || steps_per_trial < 1)
        return fail(ctx, PIC_E_INVAL, "autotune: empty candidate list or no steps");
    for (int j = 0; j < n_tiles; ++j)
        if (tiles[j] <= 0 || tiles[j] % kBlock || tiles[j] > kMaxTile)
            return fail(ctx, PIC_E_INVAL, "autotune: bad tile candidate");
    for (int j = 0; j < n_sorts; ++j)
        if (sorts[j] < 1) return fail(ctx, PIC_E_INVAL, "autotune: bad sort candidate");
    const int diag = ctx->diag_every;
    hipEvent_t ev[2] = {nullptr, nullptr};
    HIPCHK(ctx, hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return fail(ctx, PIC_E_DEVICE, "autotune: hipEventCreate");
    }
    int rc = PIC_OK;
    int best_tile = ctx->tile, best_sort = ctx->sort_every;
    double best = 1e300;
    // tiles at the current sort period; each trial starts after two steps
    // at the new tile
    for (int j = 0; j < n_tiles && rc == PIC_OK; ++j) {
        double t = 0.0;
        rc = pic_set_schedule(ctx, ctx->sort_every, diag, tiles[j]);
        if (rc == PIC_OK) rc = timed_trial(ctx, 2, steps_per_trial, ev, &t);
        if (rc == PIC_OK) {
            if (ms_out) ms_out[j] = t;
            if (t < best) {
                best = t;
                best_tile = tiles[j];
            }
        }
    }
    // sort periods at the best tile: whole periods, from a period boundary
    best = 1e300;
    for (int j = 0; j < n_sorts && rc == PIC_OK; ++j) {
        double t = 0.0;
        rc = pic_set_schedule(ctx, sorts[j], diag, best_tile);
        if (rc != PIC_OK) break;
        const int64_t to_boundary = (sorts[j] - ctx->since_sort % sorts[j]) % sorts[j];
        const int64_t periods = (steps_per_trial + sorts[j] - 1) / sorts[j];
        rc = timed_trial(ctx, (int)to_boundary, periods * sorts[j], ev, &t);
        if (rc == PIC_OK) {
            if (ms_out) ms_out[n_tiles + j] = t;
            if (t < best) {
                best = t;
                best_sort = sorts[j];
            }
        }
    }
    // the store policy of the collision kernel at the best tile and period
    bool best_nt = ctx->nt_store;
    if (rc == PIC_OK) rc = pic_set_schedule(ctx, best_sort, diag, best_tile);
    best = 1e300;
    for (int j = 0; j < 2 && rc == PIC_OK; ++j) {
        double t = 0.0;
        rc = pic_set_store_policy(ctx, j);
        if (rc != PIC_OK) break;
        const int64_t to_boundary = (best_sort - ctx->since_sort % best_sort) % best_sort;
        const int64_t periods = (steps_per_trial + best_sort - 1) / best_sort;
        rc = timed_trial(ctx, (int)to_boundary, periods * best_sort, ev, &t);
        if (rc == PIC_OK) {
            if (ms_out) ms_out[n_tiles + n_sorts + j] = t;
            if (t < best) {
                best = t;
                best_nt = j == 1;
            }
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (rc != PIC_OK) return rc;
    rc = pic_set_schedule(ctx, best_sort, diag, best_tile);
    if (rc == PIC_OK) rc = pic_set_store_policy(ctx, best_nt ? 1 : 0);
    if (rc != PIC_OK) return rc;
    if (tile_out) *tile_out = best_tile;
    if (sort_out) *sort_out = best_sort;
    return PIC_OK;
}

extern "C" int pic_reset_accumulators(pic_ctx* ctx)
{
    if (!ctx) return PIC_E_INVAL;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < ctx->n_cases; ++k) {
        const Case& C = ctx->cases_h[k];
        const size_t N = (size_t)C.n_cells;
        for (int s = 0; s < 2; ++s) {
            HIPCHK(ctx, hipMemset(C.dens_acc[s], 0, 8 * (N + 1)));
            HIPCHK(ctx, hipMemset(C.heat_acc[s], 0, 8 * N));
        }
        HIPCHK(ctx, hipMemset(C.eedf_acc, 0, 8 * (size_t)kEedfBins));
    }
    std::vector<State> st(ctx->n_cases);
    HIPCHK(ctx, hipMemcpy(st.data(), ctx->d_state, sizeof(State) * ctx->n_cases, hipMemcpyDeviceToHost));
    for (auto& s : st) s.dens_samples = s.eedf_samples = 0;
    HIPCHK(ctx, hipMemcpy(ctx->d_state, st.data(), sizeof(State) * ctx->n_cases, hipMemcpyHostToDevice));
    return PIC_OK;
}

extern "C" int pic_diagnostics(pic_ctx* ctx, int32_t case_id, uint32_t what, pic_diag* out)
{
    if (!ctx || !out || case_id < 0 || case_id >= ctx->n_cases) return PIC_E_INVAL;
    if (ctx->failed) return fail(ctx, PIC_E_STATE, ctx->err);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    Case C;
    State st;
    HIPCHK(ctx, hipMemcpy(&C, ctx->d_cases + case_id, sizeof(Case), hipMemcpyDeviceToHost));
    HIPCHK(ctx, hipMemcpy(&st, ctx->d_state + case_id, sizeof(State), hipMemcpyDeviceToHost));
    const HostCase& h = ctx->hc[case_id];
    const size_t N = (size_t)C.n_cells;
    out->step = st.step;
    out->n_particles[0] = st.n_live[0];
    out->n_particles[1] = st.n_live[1];
    out->n_slots[0] = st.n_slots[0];
    out->n_slots[1] = st.n_slots[1];
    out->vel_unit = C.dx / C.dt;
    out->acc_unit = C.dx / (C.dt * C.dt);
    if (what & PIC_DIAG_FIELDS) {
        if (out->rho) HIPCHK(ctx, hipMemcpy(out->rho, C.rho, 8 * (N + 1), hipMemcpyDefault));
        if (out->phi) HIPCHK(ctx, hipMemcpy(out->phi, C.phi, 8 * (N + 1), hipMemcpyDefault));
        if (out->E) HIPCHK(ctx, hipMemcpy(out->E, C.E, 8 * N, hipMemcpyDefault));
        if (out->chi) HIPCHK(ctx, hipMemcpy(out->chi, C.chi, 8 * N, hipMemcpyDefault));
        for (int s = 0; s < 2; ++s) {
            if (out->qfix[s]) HIPCHK(ctx, hipMemcpy(out->qfix[s], C.qfix[s], 8 * (N + 1), hipMemcpyDefault));
            if (out->cell_count[s])
                HIPCHK(ctx, hipMemcpy(out->cell_count[s], C.ccount[s], 8 * N, hipMemcpyDefault));
        }
    }
    if (what & PIC_DIAG_LEDGER) {
        HIPCHK(ctx, hipMemcpy(&out->ledger, C.history, sizeof(pic_ledger), hipMemcpyDeviceToHost));
        out->history_n = 0;
        if (out->history && out->history_cap > 0 && C.history_len > 0) {
            const int64_t have = std::min<int64_t>(st.history_n, C.history_len);
            const int64_t take = std::min<int64_t>(have, out->history_cap);
            std::vector<pic_ledger> ring((size_t)C.history_len);
            HIPCHK(ctx, hipMemcpy(ring.data(), (pic_ledger*)C.history + 1,
                                  sizeof(pic_ledger) * C.history_len, hipMemcpyDeviceToHost));
            std::vector<pic_ledger> rows((size_t)take);
            for (int64_t r = 0; r < take; ++r) {
                const int64_t idx = st.history_n - take + r;
                rows[r] = ring[(size_t)(idx % C.history_len)];
            }
            if (take > 0)
                HIPCHK(ctx, hipMemcpy(out->history, rows.data(), sizeof(pic_ledger) * take,
                                      hipMemcpyDefault));
            out->history_n = take;
        }
    }
    if (what & PIC_DIAG_STATE) {
        int rc = PIC_OK;
        for (int s = 0; s < 2; ++s) {
            const size_t ns = (size_t)st.n_slots[s];
            std::vector<int32_t> cell(ns);
            std::vector<float> off(ns), vx(ns), vy(ns), vz(ns), ab(ns);
            std::vector<uint64_t> id(ns);
            const Species& S = C.sp[s];
            if (ns) {
                HIPCHK(ctx, hipMemcpy(cell.data(), S.cell, 4 * ns, hipMemcpyDeviceToHost));
                HIPCHK(ctx, hipMemcpy(off.data(), S.off, 4 * ns, hipMemcpyDeviceToHost));
                HIPCHK(ctx, hipMemcpy(vx.data(), S.vx, 4 * ns, hipMemcpyDeviceToHost));
                std::vector<uint32_t> rr(4 * ns);
                HIPCHK(ctx, hipMemcpy(rr.data(), S.rec, 16 * ns, hipMemcpyDeviceToHost));
                for (size_t i = 0; i < ns; ++i) {
                    std::memcpy(&vy[i], &rr[4 * i + 2], 4);
                    std::memcpy(&vz[i], &rr[4 * i + 3], 4);
                    id[i] = (uint64_t)rr[4 * i] | ((uint64_t)rr[4 * i + 1] << 32);
                }
                HIPCHK(ctx, hipMemcpy(ab.data(), S.abar, 4 * ns, hipMemcpyDeviceToHost));

            }
            std::vector<uint32_t> wt(ns);
            size_t k = 0;
            // waiting-time fields are expiries of the species' clock: the
            // count left at its next move, with the capped flag
            const int ks = s == 1 ? std::max(1, (int)C.ion_sub) : 1;
            const uint32_t clk = clock_from(st.step, ks, S.n_proc > 0);
            for (size_t i = 0; i < ns; ++i) {
                if (cell[i] < 0) continue;
                const int32_t word = cell[i];
                cell[k] = word & ((1 << kCellWordBits) - 1);
                const uint32_t f = (uint32_t)word >> kCellWordBits;
                wt[k] = wait_count(f, clk) | (f & PIC_WAIT_CAPPED);
                off[k] = off[i]; vx[k] = vx[i]; vy[k] = vy[i];
                vz[k] = vz[i]; ab[k] = ab[i]; id[k] = id[i];
                ++k;
            }
            out->n_particles[s] = (int64_t)k;
            if ((int64_t)k > out->state_cap[s]) {
                rc = PIC_E_CAPACITY;
                continue;
            }
            if (k == 0) continue;
            if (out->cell[s]) HIPCHK(ctx, hipMemcpy(out->cell[s], cell.data(), 4 * k, hipMemcpyDefault));
            if (out->off[s]) HIPCHK(ctx, hipMemcpy(out->off[s], off.data(), 4 * k, hipMemcpyDefault));
            if (out->vx[s]) HIPCHK(ctx, hipMemcpy(out->vx[s], vx.data(), 4 * k, hipMemcpyDefault));
            if (out->vy[s]) HIPCHK(ctx, hipMemcpy(out->vy[s], vy.data(), 4 * k, hipMemcpyDefault));
            if (out->vz[s]) HIPCHK(ctx, hipMemcpy(out->vz[s], vz.data(), 4 * k, hipMemcpyDefault));
            if (out->id[s]) HIPCHK(ctx, hipMemcpy(out->id[s], id.data(), 8 * k, hipMemcpyDefault));
            if (out->abar[s]) HIPCHK(ctx, hipMemcpy(out->abar[s], ab.data(), 4 * k, hipMemcpyDefault));
            if (out->mcc_wait[s])
                HIPCHK(ctx, hipMemcpy(out->mcc_wait[s], wt.data(), 4 * k, hipMemcpyDefault));
        }
        if (rc) return fail(ctx, rc, "state buffers too small");
    }
    if (what & PIC_DIAG_DENSITY) {
        out->density_samples = st.dens_samples;
        for (int s = 0; s < 2; ++s) {
            if (!out->density[s]) continue;
            std::vector<long long> acc(N + 1);
            HIPCHK(ctx, hipMemcpy(acc.data(), C.dens_acc[s], 8 * (N + 1), hipMemcpyDeviceToHost));
            std::vector<double> d(N + 1);
            const std::vector<double>& cw = h.cell_w;
            for (size_t g = 0; g <= N; ++g) {
                double vol = (C.bc == PIC_BC_DIRICHLET_RF && (g == 0 || g == N)) ? 0.5 : 1.0;
                if (!cw.empty()) {
                    // node volume in units of dx: half of each adjacent cell
                    const double wl = g > 0 ? cw[g - 1] : 0.0, wr = g < N ? cw[g] : 0.0;
                    vol = 0.5 * (wl + wr) / C.dx;
                }
                d[g] = st.dens_samples > 0
                           ? (double)acc[g] / kFixScale * C.sp[s].dens_unit / vol / st.dens_samples
                           : 0.0;
            }
            HIPCHK(ctx, hipMemcpy(out->density[s], d.data(), 8 * (N + 1), hipMemcpyDefault));
        }
    }
    if (what & PIC_DIAG_HEATING) {
        for (int s = 0; s < 2; ++s)
            if (out->heating[s]) HIPCHK(ctx, hipMemcpy(out->heating[s], C.heat_acc[s], 8 * N, hipMemcpyDefault));
    }
    if (what & PIC_DIAG_EEDF) {
        out->eedf_bins = kEedfBins;
        out->eedf_bin_eV = 1.0 / C.sp[0].eedf_scale;
        out->eedf_samples = st.eedf_samples;
        if (out->eedf) HIPCHK(ctx, hipMemcpy(out->eedf, C.eedf_acc, 8 * (size_t)kEedfBins, hipMemcpyDefault));
    }
    (void)h;
    return PIC_OK;
}

extern "C" void pic_destroy(pic_ctx* ctx) { destroy_ctx(ctx); }

// ---- internal accessors for the FP64 reference form (not part of pic.h) ----
extern "C" int pic__ctx_export(pic_ctx* ctx, void** cases_h_out, int* n_cases,
                               hipStream_t* stream, void*** fp64_slot)
{
    if (!ctx) return PIC_E_INVAL;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess ||
        hipMemcpy(ctx->cases_h.data(), ctx->d_cases, sizeof(Case) * ctx->n_cases,
                  hipMemcpyDeviceToHost) != hipSuccess)
        return PIC_E_DEVICE;
    *cases_h_out = ctx->cases_h.data();
    *n_cases = ctx->n_cases;
    *stream = ctx->stream;
    *fp64_slot = &ctx->fp64;
    return PIC_OK;
}

extern "C" int pic__ctx_case_info(pic_ctx* ctx, int32_t k, pic_case_config* cfg, double* scale,
                                  int64_t* cap)
{
    if (!ctx || k < 0 || k >= ctx->n_cases) return PIC_E_INVAL;
    *cfg = ctx->hc[k].cfg;
    for (int s = 0; s < 2; ++s) {
        scale[s] = ctx->hc[k].scale[s];
        cap[s] = ctx->hc[k].cap[s];
    }
    return PIC_OK;
}

extern "C" int pic__ctx_species_consts(pic_ctx* ctx, int32_t k, int32_t s, double* out12)
{
    if (!ctx || k < 0 || k >= ctx->n_cases || s < 0 || s > 1) return PIC_E_INVAL;
    for (int i = 0; i < 12; ++i) out12[i] = ctx->hc[k].c64[s][i];
    return PIC_OK;
}

extern "C" void** pic__ctx_fp64_slot(pic_ctx* ctx) { return ctx ? &ctx->fp64 : nullptr; }

extern "C" int pic__ctx_table(pic_ctx* ctx, int32_t s, int32_t p, int32_t* n,
                              const double** sigma)
{
    if (!ctx || s < 0 || s > 1 || p < 0 || p >= (int)ctx->sigma[s].size()) return PIC_E_INVAL;
    *n = (int32_t)ctx->sigma[s][p].size();
    *sigma = ctx->sigma[s][p].data();
    return PIC_OK;
}

extern "C" const char* pic_last_error(const pic_ctx* ctx)
{
    if (!ctx) return "null context";
    return ctx->err.c_str();
}
