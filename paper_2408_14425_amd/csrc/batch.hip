// batch.hip -- formal solutions of many atmospheres and wavelength batches
// (the radiance-cascades formal solution of Osborne & Sannikov,
// arXiv:2408.14425, Secs. 2.3 and 3.2), batched.
//
// Work item = (atmosphere, 16-wavelength batch, cascade, probe tile). Each
// atmosphere has a few buffer slots (a pair of cascade buffers each); batch
// b uses slot b mod K and runs in round b div K. A generation is the set of
// items with the same (round, distance from the atmosphere's top cascade):
// every dependency of an item (the cascade above of the same batch, or the
// last cascade of the batch that used the slot before) lies in an earlier
// generation, so one grouped launch per generation, in stream order, needs
// no waiting between workgroups. Within a launch the workgroups take items
// in order; each marches its probe tile with the same march_ray as the
// per-level kernels. Cascade 0 writes J directly. The whole sequence (input
// prep for every atmosphere + all generations) is captured into a HIP graph
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
    const float* scale_b;
    const float* inv_scale_b;
    float* J;
    int32_t lam0, n_valid;
    int64_t ncell;
    int32_t dep;      // task this one waits for, or -1
    uint32_t n_items;
    int32_t level;
    int32_t tx, tz;   // probe tile
};

struct Item {
    int32_t task;
    int32_t u0, v0;
};

constexpr int32_t kMaxSlots = 4;

// One generation: workgroup g processes items begin + g, begin + g + grid, ...
template <bool F16>
__global__ __launch_bounds__(kBlock) void k_batch_gen(const Task* __restrict__ tasks, const Item* __restrict__ items,
                                                      uint32_t begin, uint32_t end)
{
    __shared__ uint4 seg[kBlock / 64][4][16];
    const march::RowCtx c = march::row_ctx();
    {
        uint4* sw = &seg[c.w][0][0];
        sw[c.lane] = make_uint4(0u, 0u, 0u, 0u);
        march::wave_sync();
    }
    for (uint32_t it = begin + blockIdx.x; it < end; it += gridDim.x) {
        const Item item = items[it];
        const Task& T = tasks[item.task];
        march::FieldOp op{};
        op.Fb = T.Fb;
        op.fb_bytes = T.fb_bytes;
        op.init(c.l);
        const int32_t N = T.L.nd;
        const int64_t n_rays = (int64_t)T.tx * T.tz * N;
        for (int64_t base = (int64_t)c.w * 4; base < n_rays; base += march::kRaysPerBlock) {
            const int64_t r = base + c.row;
            const int32_t k = (int32_t)(r % N);
            const int32_t pl = (int32_t)(r / N);
            const int32_t u = item.u0 + pl % T.tx, v = item.v0 + pl / T.tx;
            const bool active = r < n_rays && u < T.L.px && v < T.L.pz;
            const int64_t ray = ((int64_t)v * T.L.px + u) * N + k;
            if (F16) {
                march::UpF16 up{(const __half*)T.up, T.inv_scale_b, 0.0f};
                up.init(c.l);
                if (T.level == 0) {
                    march::JEpi epi{T.J, T.lam0, T.n_valid, T.ncell};
                    march::march_ray(T.L, T.nx, T.nz, op, epi, T.dirs, up, seg[c.w], nullptr, c, ray, u, v, k, active);
                } else {
                    march::StoreF16Epi epi{(__half*)T.out, T.scale_b, 0.0f};
                    epi.init(c.l);
                    march::march_ray(T.L, T.nx, T.nz, op, epi, T.dirs, up, seg[c.w], nullptr, c, ray, u, v, k, active);
                }
            } else {
                march::UpF32 up{(const float*)T.up};
                if (T.level == 0) {
                    march::JEpi epi{T.J, T.lam0, T.n_valid, T.ncell};
                    march::march_ray(T.L, T.nx, T.nz, op, epi, T.dirs, up, seg[c.w], nullptr, c, ray, u, v, k, active);
                } else {
                    march::StoreEpi epi{(float*)T.out};
                    march::march_ray(T.L, T.nx, T.nz, op, epi, T.dirs, up, seg[c.w], nullptr, c, ray, u, v, k, active);
                }
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
    std::vector<float*> scale, inv_scale;
    std::vector<void*> casc;          // per (atmosphere, slot): 2 buffers back to back
    std::vector<size_t> casc_half;     // bytes of one of the two buffers
    std::vector<int32_t> casc_index;   // first slot of atmosphere a
    std::vector<int32_t> n_slots;      // slots of atmosphere a
    int32_t rays_per_item = 4096;
    std::vector<Task> tasks_h;
    std::vector<Item> items_h;
    Task* tasks_d = nullptr;
    Item* items_d = nullptr;
    size_t tasks_cap = 0, items_cap = 0;
    std::vector<uint32_t> gen_begin;  // item range of each generation: [gen_begin[g], gen_begin[g + 1])
    int grid_cap = 0;                 // workgroups per launch at most (resident capacity)
    std::vector<float*> J_bound;  // J pointers the tasks were built for
    // graph
    bool use_graph = true;
    hipStream_t cap = nullptr;  // capture stream (the legacy default stream cannot be captured)
    hipGraphExec_t gexec = nullptr;
    std::vector<const float*> g_chi, g_eta;
    std::vector<void*> allocs;
};

namespace {

int32_t bfail(int32_t c, const std::string& m) { return rcx::fail(c, m); }

template <class P>
hipError_t balloc(rcx_batch* s, P** p, size_t bytes)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) s->allocs.push_back(q);
    *p = (P*)q;
    return e;
}

// Probe tile with about `rays` rays for a cascade of N directions.
void tile_for(int32_t rays, int32_t N, int32_t px, int32_t pz, int32_t* tx, int32_t* tz)
{
    int64_t probes = std::max<int64_t>(1, rays / N);
    int32_t a = 1;
    while ((int64_t)(a * 2) * (a * 2) <= probes) a *= 2;
    int32_t b = a;
    if ((int64_t)a * b * 2 <= probes) b *= 2;
    *tx = std::min(b, px);
    *tz = std::min(a, pz);
}

// Build the task and item lists for the current J pointers and tile size,
// grouped into generations. Returns false if a dependency would not precede
// its dependent (an internal error).
bool build_work(rcx_batch* s, float* const* J)
{
    s->tasks_h.clear();
    s->items_h.clear();
    struct Pending {
        int32_t round, top_dist, task;
    };
    std::vector<Pending> order;
    for (int32_t a = 0; a < s->n_atm; ++a) {
        const rcx_plan* P = s->plans[a];
        const int64_t ncell = (int64_t)P->grid.nx * P->grid.nz;
        const int32_t K = s->n_slots[a];
        std::vector<int32_t> last(s->n_batch[a], -1);  // cascade-0 task of each batch
        for (int32_t b = 0; b < s->n_batch[a]; ++b) {
            const int32_t slot = s->casc_index[a] + b % K;
            char* buf0 = (char*)s->casc[slot];
            char* bufs[2] = {buf0, buf0 + s->casc_half[slot]};
            int cur = 0;
            int32_t prev = -1;
            const void* up = nullptr;
            for (int32_t i = P->n_casc - 1; i >= 0; --i) {
                if (P->top_skipped && i == P->n_casc - 1) continue;
                const LevelDesc& L = P->levels[i];
                Task T{};
                T.L = L;
                T.nx = P->grid.nx;
                T.nz = P->grid.nz;
                T.dirs = P->dirs_dev + P->dir_off[i];
                T.Fb = s->F[a] + (size_t)b * ncell * kLB;
                T.fb_bytes = (uint32_t)(ncell * kLB * sizeof(float2));
                T.up = L.has_up ? up : nullptr;
                T.out = bufs[cur];
                T.scale_b = s->f16 ? s->scale[a] + b * kLB : nullptr;
                T.inv_scale_b = s->f16 ? s->inv_scale[a] + b * kLB : nullptr;
                T.J = J ? J[a] : nullptr;
                T.lam0 = b * kLB;
                T.n_valid = std::min(kLB, s->n_wave[a] - b * kLB);
                T.ncell = ncell;
                // the cascade above, or for the batch's first cascade the
                // batch that used this slot before
                T.dep = L.has_up ? prev : (prev < 0 && b >= K ? last[b - K] : -1);
                T.level = i;
                tile_for(s->rays_per_item, L.nd, L.px, L.pz, &T.tx, &T.tz);
                const int32_t ntx = (L.px + T.tx - 1) / T.tx, ntz = (L.pz + T.tz - 1) / T.tz;
                T.n_items = (uint32_t)ntx * ntz;
                const int32_t ti = (int32_t)s->tasks_h.size();
                s->tasks_h.push_back(T);
                order.push_back({b / K, P->n_casc - 1 - i, ti});
                prev = ti;
                up = bufs[cur];
                cur ^= 1;
            }
            last[b] = prev;
        }
    }
    // Slot rounds, then top-down; among equal keys larger tasks first (they
    // bound the makespan). Every dependency sorts strictly earlier.
    std::stable_sort(order.begin(), order.end(), [&](const Pending& x, const Pending& y) {
        if (x.round != y.round) return x.round < y.round;
        if (x.top_dist != y.top_dist) return x.top_dist < y.top_dist;
        const Task& a = s->tasks_h[x.task];
        const Task& b = s->tasks_h[y.task];
        return (int64_t)a.L.px * a.L.pz * a.L.nd > (int64_t)b.L.px * b.L.pz * b.L.nd;
    });
    s->gen_begin.clear();
    std::vector<int32_t> gen_of(s->tasks_h.size(), -1);
    for (size_t q = 0; q < order.size(); ++q) {
        const auto& o = order[q];
        if (q == 0 || o.round != order[q - 1].round || o.top_dist != order[q - 1].top_dist)
            s->gen_begin.push_back((uint32_t)s->items_h.size());
        gen_of[o.task] = (int32_t)s->gen_begin.size() - 1;
        const Task& T = s->tasks_h[o.task];
        for (int32_t v0 = 0; v0 < T.L.pz; v0 += T.tz)
            for (int32_t u0 = 0; u0 < T.L.px; u0 += T.tx) s->items_h.push_back({o.task, u0, v0});
    }
    s->gen_begin.push_back((uint32_t)s->items_h.size());
    // every dependency lies in an earlier generation
    for (size_t t = 0; t < s->tasks_h.size(); ++t) {
        const Task& T = s->tasks_h[t];
        if (gen_of[t] < 0) return false;
        if (T.dep >= 0 && !(gen_of[T.dep] >= 0 && gen_of[T.dep] < gen_of[t])) return false;
    }
    return true;
}

hipError_t upload_work(rcx_batch* s)
{
    hipError_t e = hipSuccess;
    if (s->tasks_h.size() > s->tasks_cap) {
        if (s->tasks_d) (void)hipFree(s->tasks_d);
        s->tasks_cap = s->tasks_h.size();
        e = hipMalloc(&s->tasks_d, sizeof(Task) * s->tasks_cap);
        if (e != hipSuccess) return e;
    }
    if (s->items_h.size() > s->items_cap) {
        if (s->items_d) (void)hipFree(s->items_d);
        s->items_cap = s->items_h.size();
        e = hipMalloc(&s->items_d, sizeof(Item) * s->items_cap);
        if (e != hipSuccess) return e;
    }
    e = hipMemcpy(s->tasks_d, s->tasks_h.data(), sizeof(Task) * s->tasks_h.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(s->items_d, s->items_h.data(), sizeof(Item) * s->items_h.size(), hipMemcpyHostToDevice);
    return e;
}

// Enqueue one batch solve (no synchronisation).
hipError_t enqueue(rcx_batch* s, const float* const* chi, const float* const* eta, hipStream_t st)
{
    for (int32_t a = 0; a < s->n_atm; ++a) {
        const rcx_plan* P = s->plans[a];
        const int64_t ncell = (int64_t)P->grid.nx * P->grid.nz;
        hipError_t e = launch_prep(chi[a], eta[a], s->F[a], s->n_wave[a], ncell, (float)P->grid.voxel_scale,
                                   s->f16 ? s->smax[a] : nullptr, st);
        if (e == hipSuccess && s->f16) e = launch_scales(s->n_batch[a] * kLB, s->smax[a], s->scale[a], s->inv_scale[a], st);
        if (e != hipSuccess) return e;
    }
    for (size_t g = 0; g + 1 < s->gen_begin.size(); ++g) {
        const uint32_t b = s->gen_begin[g], e = s->gen_begin[g + 1];
        const unsigned grid = (unsigned)std::min<uint32_t>(e - b, (uint32_t)s->grid_cap);
        if (s->f16)
            hipLaunchKernelGGL(k_batch_gen<true>, dim3(grid), dim3(kBlock), 0, st, s->tasks_d, s->items_d, b, e);
        else
            hipLaunchKernelGGL(k_batch_gen<false>, dim3(grid), dim3(kBlock), 0, st, s->tasks_d, s->items_d, b, e);
        hipError_t r = hipGetLastError();
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

void drop_graph(rcx_batch* s)
{
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
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
    rcx_batch* s = new (std::nothrow) rcx_batch();
    if (!s) return bfail(RCX_E_NOMEM, "rcx_batch_create: host allocation");
    s->n_atm = n_atm;
    s->f16 = p->storage == RCX_STORE_F16_SCALED;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (r != hipSuccess && e == hipSuccess) e = r;
    };
    for (int32_t a = 0; a < n_atm; ++a) {
        rcx_plan* P = nullptr;
        rcx_params pa = *p;
        int32_t rc = rcx_plan_create(&grids[a], &pa, kLB, &P);
        if (rc != RCX_OK) {
            rcx_batch_destroy(s);
            return rc;
        }
        // the batch keeps its own buffers; the plan's own workspace is not needed
        if (P->ws_own) {
            (void)hipFree(P->ws_own);
            P->ws_own = nullptr;
        }
        s->plans.push_back(P);
        if (n_wave[a] < 1) {
            rcx_batch_destroy(s);
            return bfail(RCX_E_INVALID, "rcx_batch_create: n_wave must be positive");
        }
        s->n_wave.push_back(n_wave[a]);
        const int32_t nb = (n_wave[a] + kLB - 1) / kLB;
        s->n_batch.push_back(nb);
        const int64_t ncell = (int64_t)grids[a].nx * grids[a].nz;
        float2* F = nullptr;
        chk(balloc(s, &F, sizeof(float2) * ncell * nb * kLB));
        s->F.push_back(F);
        unsigned int* sm = nullptr;
        float *sc = nullptr, *isc = nullptr;
        chk(balloc(s, &sm, sizeof(unsigned int) * nb * kLB));
        chk(balloc(s, &sc, sizeof(float) * nb * kLB));
        chk(balloc(s, &isc, sizeof(float) * nb * kLB));
        s->smax.push_back(sm);
        s->scale.push_back(sc);
        s->inv_scale.push_back(isc);
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
    chk(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
    if (e != hipSuccess) {
        rcx_batch_destroy(s);
        return bfail(RCX_E_NOMEM, std::string("rcx_batch_create: hipMalloc: ") + hipGetErrorName(e));
    }
    // workgroups per generation launch: at most the resident capacity
    int dev = 0, n_cu = 0, per_cu = 0;
    chk(hipGetDevice(&dev));
    chk(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    if (s->f16)
        chk(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_gen<true>, kBlock, 0));
    else
        chk(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_gen<false>, kBlock, 0));
    if (e != hipSuccess || n_cu < 1 || per_cu < 1) {
        rcx_batch_destroy(s);
        return rcx::hip_fail(e == hipSuccess ? hipErrorInvalidValue : e, "rcx_batch_create: occupancy query");
    }
    s->grid_cap = n_cu * per_cu;
    *out = s;
    return RCX_OK;
}

int32_t rcx_batch_set_tiling(rcx_batch* s, int32_t rays_per_item)
{
    if (!s || rays_per_item < 16) return bfail(RCX_E_INVALID, "rcx_batch_set_tiling: bad argument");
    s->rays_per_item = rays_per_item;
    s->J_bound.clear();  // rebuild the work lists on the next solve
    drop_graph(s);
    return RCX_OK;
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
    const bool same_J = (int32_t)s->J_bound.size() == s->n_atm &&
                        std::equal(s->J_bound.begin(), s->J_bound.end(), J_host);
    if (!same_J) {
        if (!build_work(s, J_host)) return bfail(RCX_E_INVALID, "rcx_batch_solve: internal: work queue out of order");
        RCX_HIP_TRY(upload_work(s));
        s->J_bound.assign(J_host, J_host + s->n_atm);
        drop_graph(s);
    }
    if (s->use_graph) {
        const bool same_in = s->gexec && std::equal(s->g_chi.begin(), s->g_chi.end(), chi_host) &&
                             std::equal(s->g_eta.begin(), s->g_eta.end(), eta_host);
        if (!same_in) {
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
    RCX_HIP_TRY(hipStreamSynchronize(st));
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

int32_t rcx_batch_autotune(rcx_batch* s, const float* const* chi, const float* const* eta, float* const* J,
                           const char* cache_path, int32_t* best_rays_host, hipStream_t st)
{
    if (!s || !chi || !eta || !J || !best_rays_host) return bfail(RCX_E_INVALID, "rcx_batch_autotune: null argument");
    // cache key: the batch's shapes
    std::ostringstream key;
    key << (s->f16 ? "f16" : "f32");
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
                if (r >= 16) {
                    *best_rays_host = r;
                    return rcx_batch_set_tiling(s, r);
                }
            }
        }
    }
    const int32_t cands[] = {1024, 4096, 16384, 65536};
    double best_ms = 1e300;
    int32_t best = cands[0];
    const bool g = s->use_graph;
    s->use_graph = false;
    for (int32_t cnd : cands) {
        int32_t rc = rcx_batch_set_tiling(s, cnd);
        if (rc != RCX_OK) return rc;
        rc = rcx_batch_solve(s, chi, eta, J, st);  // warm-up and work-list build
        if (rc != RCX_OK) return rc;
        const auto t0 = std::chrono::steady_clock::now();
        rc = rcx_batch_solve(s, chi, eta, J, st);
        if (rc != RCX_OK) return rc;
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
    return rcx_batch_set_tiling(s, best);
}

int32_t rcx_batch_destroy(rcx_batch* s)
{
    if (!s) return RCX_OK;
    drop_graph(s);
    for (void* p : s->allocs) (void)hipFree(p);
    if (s->tasks_d) (void)hipFree(s->tasks_d);
    if (s->items_d) (void)hipFree(s->items_d);
    for (rcx_plan* P : s->plans) rcx_plan_destroy(P);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    delete s;
    return RCX_OK;
}

}  // extern "C"
