// batch.hip -- formal solutions of many atmospheres and wavelength batches
// (the radiance-cascades formal solution of Osborne & Sannikov,
// arXiv:2408.14425, Secs. 2.3 and 3.2), batched.
//
// Task = (atmosphere, 16-wavelength batch, cascade); the tasks of one
// (atmosphere, batch) form a chain from the top cascade down. Each
// atmosphere has a few buffer slots (a pair of cascade buffers each); chain
// b uses slot b mod K. Launches are formed by a list schedule: a set of
// active chains advances one cascade per launch, and chains are activated
// (in order, at most K per atmosphere) until a launch holds enough rays to
// fill the GPU, so small atmospheres share launches. An atmosphere whose
// every cascade fills the GPU alone gains nothing from sharing and runs
// through its plan's own solve instead (the per-cascade path, with two
// wavelength batches per lane below 256 directions), inside the same
// captured sequence. Every
// dependency (the cascade above in the same chain, or the chain that used
// the slot before) lies in an earlier launch, and stream order provides it:
// no workgroup waits on another. A launch sweeps the concatenated rays of
// its tasks, each in the same order as the per-cascade kernels, with the
// same march_ray. Cascade 0 writes J directly. The whole sequence (input
// prep for every atmosphere + all launches) is captured into a HIP graph
// and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "march_rows.h"

namespace rcx {
namespace bt {

using march::kBlock;
using march::kLB;

struct Task {
    LevelDesc L;
    int32_t nx, nz;
    const double4* dirs;
    const float2* Fb;
    uint32_t fb_bytes;
    const void* up;
    void* out;
    const int32_t* ebias_b;
    float* J;
    int32_t lam0, n_valid;
    int64_t ncell;
    int32_t dep;      // task this one depends on, or -1
    int32_t level;
    int64_t ray0;     // first ray of the task in its generation's sweep
    int64_t n_rays;   // rays the task launches (level_launch_rays, a multiple of 4)
};

constexpr int32_t kMaxSlots = 4;

// One generation: tasks [t0, t0 + nt) sorted by ray0, total rays in all.
// Grid-stride over the rays like the per-cascade kernel; the 4 rays of a
// wavefront belong to one task (every task's ray count is a multiple of 4).
template <bool F16>
__global__ __launch_bounds__(kBlock) void k_batch_gen(const Task* __restrict__ tasks, int32_t t0, int32_t nt,
                                                      int64_t total)
{
    __shared__ uint4 seg[kBlock / 64][4][march::kSegRow];
    const march::RowCtx c = march::row_ctx();
    {
        seg[c.w][c.row][c.l] = make_uint4(0u, 0u, 0u, 0u);
        march::wave_sync();
    }
    const unsigned lb = march::xcd_block_chunked(blockIdx.x, gridDim.x);
    const int64_t stride = (int64_t)gridDim.x * march::kRaysPerBlock;
    for (int64_t base = ((int64_t)lb * (kBlock / 64) + c.w) * 4; base < total; base += stride) {
        // the task holding ray `base` (the same for the whole wavefront:
        // made explicit so the descriptor is read with scalar loads)
        const int64_t wbase = (int64_t)__builtin_amdgcn_readfirstlane((int)(base >> 32)) << 32 |
                              (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)base);
        int32_t lo = t0, hi = t0 + nt - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (tasks[mid].ray0 <= wbase) lo = mid;
            else hi = mid - 1;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        const Task T = tasks[lo];  // by value: kept in registers for the march
        const int64_t rr = wbase - T.ray0 + c.row;  // < T.n_rays
        const LevelDesc L = T.L;
        // probe and direction in the task's launch order (dense, tiled, or
        // the flagged-probe list of a sparse atmosphere)
        int32_t k, u, v;
        bool active;
        march::ray_coords(L, rr, T.n_rays, k, u, v, active);
        const int64_t ray = ((int64_t)v * L.px + u) * L.nd + k;
        march::FieldOp op{};
        op.Fb = T.Fb;
        op.fb_bytes = T.fb_bytes;
        op.init(c.l);
        if (F16) {
            march::UpF16 up{(const uint16_t*)T.up, T.ebias_b};
            up.init(c.l);
            if (T.level == 0) {
                march::JEpi epi{T.J, T.lam0, T.n_valid, T.ncell};
                march::march_ray(L, T.nx, T.nz, op, epi, T.dirs, up, seg[c.w], nullptr, c, ray, u, v, k, active);
            } else {
                march::StoreF16Epi epi{(uint16_t*)T.out, T.ebias_b};
                epi.init(c.l);
                march::march_ray(L, T.nx, T.nz, op, epi, T.dirs, up, seg[c.w], nullptr, c, ray, u, v, k, active);
            }
        } else {
            march::UpF32 up{(const float*)T.up};
            if (T.level == 0) {
                march::JEpi epi{T.J, T.lam0, T.n_valid, T.ncell};
                march::march_ray(L, T.nx, T.nz, op, epi, T.dirs, up, seg[c.w], nullptr, c, ray, u, v, k, active);
            } else {
                march::StoreEpi epi{(float*)T.out};
                march::march_ray(L, T.nx, T.nz, op, epi, T.dirs, up, seg[c.w], nullptr, c, ray, u, v, k, active);
            }
        }
    }
}

}  // namespace bt
}  // namespace rcx

using namespace rcx;
using namespace rcx::bt;

struct rcx_batch {
    int32_t n_atm = 0;
    bool f16 = false;
    std::vector<rcx_plan*> plans;
    std::vector<int32_t> n_wave, n_batch;
    std::vector<float2*> F;        // per atmosphere [n_batch][ncell][16]
    std::vector<unsigned int*> smax;
    std::vector<int32_t*> ebias;
    std::vector<void*> casc;          // per (atmosphere, slot): 2 buffers back to back
    std::vector<size_t> casc_half;     // bytes of one of the two buffers
    std::vector<int32_t> casc_index;   // first slot of atmosphere a
    std::vector<int32_t> n_slots;      // slots of atmosphere a
    int64_t fill_rays = 1 << 19;      // rays a launch gathers before it stops activating chains
    std::vector<Task> tasks_h;        // grouped by generation, each group sorted by ray0
    Task* tasks_d = nullptr;
    size_t tasks_cap = 0;
    std::vector<int32_t> gen_task;    // task range of each generation: [gen_task[g], gen_task[g + 1])
    std::vector<int64_t> gen_rays;    // rays of each generation
    std::vector<float*> J_bound;  // J pointers the tasks were built for
    // atmospheres large enough to fill the GPU with every one of their
    // launches run through their plan's own solve (rcx::plan_enqueue_solve:
    // the per-cascade path, two wavelength batches per lane below 256
    // directions); the rest are list-scheduled
    std::vector<char> solo;
    int64_t solo_march = 0;  // march launches the solo atmospheres enqueued in the last solve
    // graph
    bool use_graph = true;
    hipStream_t cap = nullptr;  // capture stream (the legacy default stream cannot be captured)
    hipGraphExec_t gexec = nullptr;
    std::vector<const float*> g_chi, g_eta;
    unsigned int* flag = nullptr;  // input check (RCX_FLAG_CHECK_INPUT)
    bool check_input = false;
    std::vector<void*> allocs;
};

namespace {

int32_t bfail(int32_t c, const std::string& m) { return rcx::fail(c, m); }

// Cascades whose launch order rcx_batch_set_order sets (the tiled ones).
constexpr int32_t kWideDirs = 256;

template <class P>
hipError_t balloc(rcx_batch* s, P** p, size_t bytes)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) s->allocs.push_back(q);
    *p = (P*)q;
    return e;
}

// Build the task list for the current J pointers and launch order, grouped
// into launches by the list schedule. Returns false if a dependency would
// not precede its dependent (an internal error).
bool build_work(rcx_batch* s, float* const* J)
{
    // chains in order: atmosphere-major, batches in order
    struct Chain {
        int32_t atm;
        std::vector<Task> tasks;  // top cascade first
    };
    std::vector<Chain> chains;
    for (int32_t a = 0; a < s->n_atm; ++a) {
        if (s->solo[a]) continue;
        const rcx_plan* P = s->plans[a];
        const int64_t ncell = (int64_t)P->grid.nx * P->grid.nz;
        const int32_t K = s->n_slots[a];
        for (int32_t b = 0; b < s->n_batch[a]; ++b) {
            Chain ch;
            ch.atm = a;
            const int32_t slot = s->casc_index[a] + b % K;
            char* buf0 = (char*)s->casc[slot];
            char* bufs[2] = {buf0, buf0 + s->casc_half[slot]};
            int cur = 0;
            const void* up = nullptr;
            for (int32_t i = P->n_casc - 1; i >= 0; --i) {
                if (P->top_skipped && i == P->n_casc - 1) continue;
                Task T{};
                T.L = P->levels[i];  // the plan's launch order (rcx_batch_set_order sets it)
                if (!set_decode(T.L)) return false;
                T.nx = P->grid.nx;
                T.nz = P->grid.nz;
                T.dirs = P->dirs_dev + P->dir_off[i];
                T.Fb = s->F[a] + (size_t)b * ncell * kLB;
                T.fb_bytes = (uint32_t)(ncell * kLB * sizeof(float2));
                T.up = T.L.has_up ? up : nullptr;
                T.out = bufs[cur];
                T.ebias_b = s->f16 ? s->ebias[a] + b * kLB : nullptr;
                T.J = J ? J[a] : nullptr;
                T.lam0 = b * kLB;
                T.n_valid = std::min(kLB, s->n_wave[a] - b * kLB);
                T.ncell = ncell;
                T.level = i;
                T.n_rays = level_launch_rays(T.L);
                T.dep = -1;
                if (T.n_rays % 4 != 0) return false;
                ch.tasks.push_back(T);
                up = bufs[cur];
                cur ^= 1;
            }
            chains.push_back(std::move(ch));
        }
    }
    // list schedule
    s->tasks_h.clear();
    s->gen_task.clear();
    s->gen_rays.clear();
    std::vector<int32_t> active_of(s->n_atm, 0);
    struct Active {
        int32_t chain, pos;
    };
    std::vector<Active> active;
    size_t next = 0;  // first chain not yet activated
    std::vector<char> started(chains.size(), 0);
    while (next < chains.size() || !active.empty()) {
        int64_t rays = 0;
        for (const auto& a : active) rays += chains[a.chain].tasks[a.pos].n_rays;
        for (size_t c = next; c < chains.size() && rays < s->fill_rays; ++c) {
            if (started[c] || active_of[chains[c].atm] >= s->n_slots[chains[c].atm]) continue;
            // chains of one atmosphere start in order (their slots rotate)
            bool earlier_waiting = false;
            for (size_t d = next; d < c; ++d)
                if (!started[d] && chains[d].atm == chains[c].atm) earlier_waiting = true;
            if (earlier_waiting) continue;
            started[c] = 1;
            ++active_of[chains[c].atm];
            active.push_back({(int32_t)c, 0});
            rays += chains[c].tasks[0].n_rays;
        }
        while (next < chains.size() && started[next]) ++next;
        if (active.empty()) return false;  // cannot happen: some chain can always start
        // one launch: the next task of every active chain, larger first
        std::vector<Task> gen;
        for (auto& a : active) gen.push_back(chains[a.chain].tasks[a.pos]);
        std::stable_sort(gen.begin(), gen.end(), [](const Task& x, const Task& y) { return x.n_rays > y.n_rays; });
        s->gen_task.push_back((int32_t)s->tasks_h.size());
        int64_t ray0 = 0;
        for (Task T : gen) {
            T.ray0 = ray0;
            ray0 += T.n_rays;
            s->tasks_h.push_back(T);
        }
        s->gen_rays.push_back(ray0);
        // advance; retire finished chains
        std::vector<Active> still;
        for (auto a : active) {
            if (++a.pos < (int32_t)chains[a.chain].tasks.size()) still.push_back(a);
            else --active_of[chains[a.chain].atm];
        }
        active.swap(still);
    }
    s->gen_task.push_back((int32_t)s->tasks_h.size());
    // Check: the task that wrote a task's input cascade (same batch, the
    // cascade above) sits in an earlier launch, and no task in between
    // overwrote that buffer.
    std::vector<int32_t> gen_of(s->tasks_h.size());
    for (size_t g = 0; g + 1 < s->gen_task.size(); ++g)
        for (int32_t t = s->gen_task[g]; t < s->gen_task[g + 1]; ++t) gen_of[t] = (int32_t)g;
    for (size_t t = 0; t < s->tasks_h.size(); ++t) {
        const Task& T = s->tasks_h[t];
        if (!T.up) continue;
        int32_t writer = -1;
        for (size_t w = 0; w < s->tasks_h.size(); ++w)
            if (s->tasks_h[w].level == T.level + 1 && s->tasks_h[w].lam0 == T.lam0 && s->tasks_h[w].Fb == T.Fb)
                writer = (int32_t)w;
        if (writer < 0 || s->tasks_h[writer].out != T.up || !(gen_of[writer] < gen_of[t])) return false;
        for (size_t w = 0; w < s->tasks_h.size(); ++w)
            if ((int32_t)w != writer && s->tasks_h[w].out == T.up && gen_of[w] >= gen_of[writer] && gen_of[w] <= gen_of[t])
                return false;
    }
    return true;
}

hipError_t upload_work(rcx_batch* s)
{
    if (s->tasks_h.empty()) return hipSuccess;  // every atmosphere runs through its plan
    if (s->tasks_h.size() > s->tasks_cap) {
        if (s->tasks_d) (void)hipFree(s->tasks_d);
        s->tasks_d = nullptr;
        s->tasks_cap = s->tasks_h.size();
        hipError_t e = hipMalloc(&s->tasks_d, sizeof(Task) * s->tasks_cap);
        if (e != hipSuccess) return e;
    }
    return hipMemcpy(s->tasks_d, s->tasks_h.data(), sizeof(Task) * s->tasks_h.size(), hipMemcpyHostToDevice);
}

// Enqueue one batch solve (no synchronisation).
hipError_t enqueue(rcx_batch* s, const float* const* chi, const float* const* eta, hipStream_t st)
{
    s->solo_march = 0;
    for (int32_t a = 0; a < s->n_atm; ++a) {
        if (!s->solo[a]) continue;
        int64_t n = 0;
        if (plan_enqueue_solve(s->plans[a], s->n_wave[a], chi[a], eta[a], s->J_bound[a], st, &n) != RCX_OK)
            return hipErrorInvalidValue;
        s->solo_march += n;
    }
    for (int32_t a = 0; a < s->n_atm; ++a) {
        if (s->solo[a]) continue;
        const rcx_plan* P = s->plans[a];
        const int64_t ncell = (int64_t)P->grid.nx * P->grid.nz;
        hipError_t e = launch_prep(chi[a], eta[a], s->F[a], s->n_wave[a], ncell, (float)P->grid.voxel_scale,
                                   s->f16 ? s->smax[a] : nullptr, st);
        if (e == hipSuccess && s->f16) e = launch_ebias(s->n_batch[a] * kLB, s->smax[a], s->ebias[a], st);
        // sparse atmosphere: unflagged cells transparent and empty
        if (e == hipSuccess && P->mask_dev) e = launch_mask_fields(s->F[a], P->mask_dev, ncell, s->n_batch[a], st);
        if (e != hipSuccess) return e;
    }
    for (size_t g = 0; g + 1 < s->gen_task.size(); ++g) {
        const int32_t t0 = s->gen_task[g], nt = s->gen_task[g + 1] - t0;
        const int64_t total = s->gen_rays[g];
        const dim3 grid = march_grid(total);
        if (s->f16)
            hipLaunchKernelGGL(k_batch_gen<true>, grid, dim3(kBlock), 0, st, s->tasks_d, t0, nt, total);
        else
            hipLaunchKernelGGL(k_batch_gen<false>, grid, dim3(kBlock), 0, st, s->tasks_d, t0, nt, total);
        hipError_t r = hipGetLastError();
        if (r != hipSuccess) return r;
    }
    // sparse atmospheres: J = 0 at unflagged cells
    for (int32_t a = 0; a < s->n_atm; ++a) {
        const rcx_plan* P = s->plans[a];
        if (s->solo[a] || !P->mask_dev) continue;
        hipError_t e = launch_mask_j(s->J_bound[a], P->mask_dev, (int64_t)P->grid.nx * P->grid.nz, s->n_wave[a], st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Solves run asynchronously: before the work list, the graph or a plan's
// lists change, the device must have finished any solve still reading them.
void drop_graph(rcx_batch* s)
{
    if (s->gexec) {
        (void)hipDeviceSynchronize();
        (void)hipGraphExecDestroy(s->gexec);
    }
    s->gexec = nullptr;
}

}  // namespace

extern "C" {

int32_t rcx_batch_create(int32_t n_atm, const rcx_grid* grids, const int32_t* n_wave, const rcx_params* p,
                         rcx_batch** out)
{
    if (out) *out = nullptr;
    if (n_atm < 1 || !grids || !n_wave || !p || !out) return bfail(RCX_E_INVALID, "rcx_batch_create: bad argument");
    if (p->c0_dirs != 4) return bfail(RCX_E_UNSUPPORTED, "rcx_batch_create: the fused J epilogue needs c0_dirs = 4");
    if (p->n_cascades != 0) return bfail(RCX_E_UNSUPPORTED, "rcx_batch_create: cascades are chosen per atmosphere");
    if (p->n_incl != 1) return bfail(RCX_E_UNSUPPORTED, "rcx_batch_create: flatland only (n_incl = 1)");
    if ((p->flags & ~RCX_FLAG_CHECK_INPUT) != 0)
        return bfail(RCX_E_UNSUPPORTED, "rcx_batch_create: only RCX_FLAG_CHECK_INPUT (basic merge only)");
    rcx_batch* s = new (std::nothrow) rcx_batch();
    if (!s) return bfail(RCX_E_NOMEM, "rcx_batch_create: host allocation");
    s->n_atm = n_atm;
    s->f16 = p->storage == RCX_STORE_F16_SCALED;
    s->check_input = (p->flags & RCX_FLAG_CHECK_INPUT) != 0;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (r != hipSuccess && e == hipSuccess) e = r;
    };
    for (int32_t a = 0; a < n_atm; ++a) {
        if (n_wave[a] < 1) {
            rcx_batch_destroy(s);
            return bfail(RCX_E_INVALID, "rcx_batch_create: n_wave must be positive");
        }
        rcx_plan* P = nullptr;
        rcx_params pa = *p;
        pa.flags &= ~RCX_FLAG_CHECK_INPUT;  // the batch checks its inputs itself
        int32_t rc = rcx_plan_create(&grids[a], &pa, n_wave[a], &P);
        if (rc != RCX_OK) {
            rcx_batch_destroy(s);
            return rc;
        }
        s->plans.push_back(P);
        s->n_wave.push_back(n_wave[a]);
        const int32_t nb = (n_wave[a] + kLB - 1) / kLB;
        s->n_batch.push_back(nb);
        // every launch of this atmosphere fills the GPU on its own: its
        // plan's solve, with the plan's workspace
        bool solo = true;
        for (int32_t i = 0; i < P->n_casc; ++i) {
            if (P->top_skipped && i == P->n_casc - 1) continue;
            const LevelDesc& L = P->levels[i];
            if ((int64_t)L.px * L.pz * L.nd < s->fill_rays) solo = false;
        }
        s->solo.push_back(solo ? 1 : 0);
        if (solo) {
            s->F.push_back(nullptr);
            s->smax.push_back(nullptr);
            s->ebias.push_back(nullptr);
            s->casc_index.push_back((int32_t)s->casc.size());
            s->n_slots.push_back(0);
            continue;
        }
        // list-scheduled: the batch keeps its own buffers
        if (P->ws_own) {
            (void)hipFree(P->ws_own);
            P->ws_own = nullptr;
        }
        const int64_t ncell = (int64_t)grids[a].nx * grids[a].nz;
        float2* F = nullptr;
        chk(balloc(s, &F, sizeof(float2) * ncell * nb * kLB));
        s->F.push_back(F);
        unsigned int* sm = nullptr;
        int32_t* eb = nullptr;
        chk(balloc(s, &sm, sizeof(unsigned int) * nb * kLB));
        chk(balloc(s, &eb, sizeof(int32_t) * nb * kLB));
        s->smax.push_back(sm);
        s->ebias.push_back(eb);
        int64_t max_entries = 0;
        for (const auto& L : P->levels) max_entries = std::max<int64_t>(max_entries, (int64_t)L.px * L.pz * L.nd);
        s->casc_index.push_back((int32_t)s->casc.size());
        const int32_t K = std::min(nb, kMaxSlots);
        s->n_slots.push_back(K);
        const size_t half = ((size_t)max_entries * kLB * (s->f16 ? 2 : 4) + 255) & ~size_t(255);
        for (int32_t b = 0; b < K; ++b) {
            void* buf = nullptr;
            chk(balloc(s, &buf, 2 * half));
            s->casc.push_back(buf);
            s->casc_half.push_back(half);
        }
        if (e != hipSuccess) break;
    }
    if (s->check_input) chk(balloc(s, &s->flag, sizeof(unsigned int)));
    chk(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
    if (e != hipSuccess) {
        rcx_batch_destroy(s);
        return bfail(RCX_E_NOMEM, std::string("rcx_batch_create: hipMalloc: ") + hipGetErrorName(e));
    }
    *out = s;
    return RCX_OK;
}

int32_t rcx_batch_set_order(rcx_batch* s, int32_t tile_probes, int32_t tile_dirs)
{
    if (!s || tile_probes < 0 || tile_probes > 64) return bfail(RCX_E_INVALID, "rcx_batch_set_order: bad argument");
    RCX_HIP_TRY(hipDeviceSynchronize());  // a solve in flight reads the plans' lists
    for (rcx_plan* P : s->plans)
        for (int32_t i = 0; i < P->n_casc; ++i) {
            if (P->levels[i].nd < kWideDirs) continue;
            const int32_t rc =
                rcx_plan_set_order(P, i, tile_probes, tile_dirs, P->levels[i].xcd_chunk, P->levels[i].shared_walk);
            if (rc != RCX_OK) return rc;
        }
    s->J_bound.clear();  // rebuild the task list on the next solve (after the stream has finished)
    drop_graph(s);
    return RCX_OK;
}

int32_t rcx_batch_set_active_host(rcx_batch* s, int32_t atm, const uint8_t* active_host)
{
    if (!s || atm < 0 || atm >= s->n_atm) return bfail(RCX_E_INVALID, "rcx_batch_set_active_host: bad argument");
    RCX_HIP_TRY(hipDeviceSynchronize());  // a solve in flight reads the plan's lists
    const int32_t rc = rcx_plan_set_active_host(s->plans[atm], active_host, nullptr);
    s->J_bound.clear();  // ray counts changed: rebuild the task list on the next solve
    drop_graph(s);
    return rc;
}

int32_t rcx_batch_set_graph(rcx_batch* s, int32_t enable)
{
    if (!s) return bfail(RCX_E_INVALID, "rcx_batch_set_graph: null batch");
    s->use_graph = enable != 0;
    drop_graph(s);
    return RCX_OK;
}

int32_t rcx_batch_solve(rcx_batch* s, const float* const* chi_host, const float* const* eta_host, float* const* J_host,
                        hipStream_t st)
{
    if (!s || !chi_host || !eta_host || !J_host) return bfail(RCX_E_INVALID, "rcx_batch_solve: null argument");
    for (int32_t a = 0; a < s->n_atm; ++a)
        if (!chi_host[a] || !eta_host[a] || !J_host[a]) return bfail(RCX_E_INVALID, "rcx_batch_solve: null array");
    if (s->check_input) {
        // every atmosphere's chi and eta finite and non-negative (synchronises)
        RCX_HIP_TRY(launch_zero_flag(s->flag, st));
        for (int32_t a = 0; a < s->n_atm; ++a) {
            const int64_t n = (int64_t)s->n_wave[a] * s->plans[a]->grid.nx * s->plans[a]->grid.nz;
            RCX_HIP_TRY(launch_check_f32(chi_host[a], n, kCheckNonNegative, s->flag, st));
            RCX_HIP_TRY(launch_check_f32(eta_host[a], n, kCheckNonNegative, s->flag, st));
        }
        const int32_t rc = check_flag_result(s->flag, "rcx_batch_solve: chi or eta", st);
        if (rc != RCX_OK) return rc;
    }
    const bool same_J = (int32_t)s->J_bound.size() == s->n_atm &&
                        std::equal(s->J_bound.begin(), s->J_bound.end(), J_host);
    const bool same_in = s->gexec && std::equal(s->g_chi.begin(), s->g_chi.end(), chi_host) &&
                         std::equal(s->g_eta.begin(), s->g_eta.end(), eta_host);
    if (!same_J || (s->use_graph && !same_in)) {
        // the work list or the graph changes: a solve still in flight reads
        // them, so it must end first
        RCX_HIP_TRY(hipStreamSynchronize(st));
    }
    if (!same_J) {
        if (!build_work(s, J_host)) return bfail(RCX_E_INVALID, "rcx_batch_solve: internal: work queue out of order");
        RCX_HIP_TRY(upload_work(s));
        s->J_bound.assign(J_host, J_host + s->n_atm);
        drop_graph(s);
    }
    if (s->use_graph) {
        if (!s->gexec || !same_in) {
            drop_graph(s);
            hipGraph_t g = nullptr;
            RCX_HIP_TRY(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue(s, chi_host, eta_host, s->cap);
            hipError_t e2 = hipStreamEndCapture(s->cap, &g);
            if (e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return rcx::hip_fail(e, "rcx_batch_solve: capture");
            }
            RCX_HIP_TRY(e2);
            e = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            RCX_HIP_TRY(e);
            s->g_chi.assign(chi_host, chi_host + s->n_atm);
            s->g_eta.assign(eta_host, eta_host + s->n_atm);
        }
        RCX_HIP_TRY(hipGraphLaunch(s->gexec, st));
    } else {
        RCX_HIP_TRY(enqueue(s, chi_host, eta_host, st));
    }
    return RCX_OK;
}

int32_t rcx_batch_work(const rcx_batch* s, int64_t* rays_nonempty_host, int64_t* cell_steps_host)
{
    if (!s || !rays_nonempty_host || !cell_steps_host) return bfail(RCX_E_INVALID, "rcx_batch_work: null argument");
    int64_t r = 0, c = 0;
    for (int32_t a = 0; a < s->n_atm; ++a) {
        rcx_work w;
        int32_t rc = rcx_plan_work(s->plans[a], &w);
        if (rc != RCX_OK) return rc;
        r += w.rays_nonempty * s->n_wave[a];
        c += w.cell_steps * s->n_wave[a];
    }
    *rays_nonempty_host = r;
    *cell_steps_host = c;
    return RCX_OK;
}

int32_t rcx_batch_launches(const rcx_batch* s, int32_t* march_host, int32_t* all_host)
{
    if (!s || !march_host || !all_host) return bfail(RCX_E_INVALID, "rcx_batch_launches: null argument");
    const int32_t march = (s->gen_task.empty() ? 0 : (int32_t)s->gen_task.size() - 1) + (int32_t)s->solo_march;
    int32_t other = 0;
    if (march > 0)
        for (int32_t a = 0; a < s->n_atm; ++a) {
            other += 1 + (s->f16 ? 1 : 0);              // field prep (+ exponent bias)
            if (s->plans[a]->mask_dev) other += 2;      // masked fields, masked J
        }
    *march_host = march;
    *all_host = march + other;
    return RCX_OK;
}

int32_t rcx_batch_autotune(rcx_batch* s, const float* const* chi, const float* const* eta, float* const* J,
                           const char* cache_path, int32_t* best_rays_host, hipStream_t st)
{
    if (!s || !chi || !eta || !J || !best_rays_host) return bfail(RCX_E_INVALID, "rcx_batch_autotune: null argument");
    // cache key: the batch's shapes
    std::ostringstream key;
    key << "v2_" << (s->f16 ? "f16" : "f32");
    for (int32_t a = 0; a < s->n_atm; ++a)
        if (s->plans[a]->mask_dev) key << "_sparse" << a << "_" << s->plans[a]->levels[0].n_active;
    for (int32_t a = 0; a < s->n_atm; ++a)
        key << "_" << s->plans[a]->grid.nx << "x" << s->plans[a]->grid.nz << "w" << s->n_wave[a];
    const std::string k = key.str();
    if (cache_path) {
        std::ifstream f(cache_path);
        std::string line;
        while (std::getline(f, line)) {
            const std::string pre = "\"" + k + "\": ";
            const size_t pos = line.find(pre);
            if (pos != std::string::npos) {
                const int32_t r = std::atoi(line.c_str() + pos + pre.size());
                if (r >= 0 && r <= 64064) {
                    *best_rays_host = r;
                    return rcx_batch_set_order(s, r / 1000, r % 1000);
                }
            }
        }
    }
    // candidate (tile_probes, tile_dirs), coded tile_probes * 1000 + tile_dirs
    const int32_t cands[] = {0, 2032, 4016, 4032, 4064, 8032};
    double best_ms = 1e300;
    int32_t best = cands[0];
    const bool g = s->use_graph;
    s->use_graph = false;
    for (int32_t cnd : cands) {
        int32_t rc = rcx_batch_set_order(s, cnd / 1000, cnd % 1000);
        if (rc != RCX_OK) return rc;
        rc = rcx_batch_solve(s, chi, eta, J, st);  // warm-up and work-list build
        if (rc != RCX_OK) return rc;
        RCX_HIP_TRY(hipStreamSynchronize(st));
        const auto t0 = std::chrono::steady_clock::now();
        rc = rcx_batch_solve(s, chi, eta, J, st);
        if (rc != RCX_OK) return rc;
        RCX_HIP_TRY(hipStreamSynchronize(st));
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (ms < best_ms) {
            best_ms = ms;
            best = cnd;
        }
    }
    s->use_graph = g;
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        f << "{\"" << k << "\": " << best << ", \"ms\": " << best_ms << "}\n";
    }
    *best_rays_host = best;
    return rcx_batch_set_order(s, best / 1000, best % 1000);
}

int32_t rcx_batch_destroy(rcx_batch* s)
{
    if (!s) return RCX_OK;
    drop_graph(s);
    for (void* p : s->allocs) (void)hipFree(p);
    if (s->tasks_d) (void)hipFree(s->tasks_d);
    for (rcx_plan* P : s->plans) rcx_plan_destroy(P);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    delete s;
    return RCX_OK;
}

}  // extern "C"
