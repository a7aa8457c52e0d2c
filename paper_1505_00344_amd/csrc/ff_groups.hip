// ff_groups.hip — ragged batch of particle groups (Appendix A "Particle
// Group": each group has its own count, direction and, here, its own system)
// in one persistent launch, plus the launch-shape autotuner.
//
// The host splits every group into tiles of block*PPT particles, orders the
// groups by decreasing cost per particle (the 15-dimensional ring first) and
// passes the whole group table as kernel arguments.  Persistent blocks pull
// tile indices from an atomic counter until the table is exhausted (every
// wave reaches that exit); a tile belongs to one group, so a wavefront never
// mixes systems.  Each tile runs the same rk4_tile code as ff_integrate,
// hence the batch is bitwise equal to per-group calls.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "ff_rk4.h"

namespace ff {

namespace {

constexpr int kMaxGroups = 32;
constexpr int kMaxSys = 8;

enum Kind : int8_t { K_LORENZ = 0, K_WC = 1, K_HH1 = 2, K_HH3 = 3, K_LIN1 = 4, K_LIN2 = 5, K_LIN3 = 6, K_LIN4 = 7 };

struct GroupEntry {
    void* state;
    void* comp;
    const void* pp;
    int64_t ld;
    int32_t n;
    int32_t tile_begin;
    int8_t kind, sys, n_pp, ppt;
    int8_t slot[kMaxPP];
    double h, h2, h6;
};

struct GroupTable {
    GroupEntry g[kMaxGroups];
    ParamBlock sp[kMaxSys];
    int64_t steps;
    int32_t ngroups, ntiles;
};
static_assert(sizeof(GroupTable) <= 3800, "group table must fit the kernel-argument segment");

template <template <typename> class SysT, typename R, bool KAHAN, int PPT>
__device__ __forceinline__ void run_tile(const GroupTable& tab, const GroupEntry& e, int t) {
    RK4Args a;
    a.state = e.state;
    a.comp = e.comp;
    a.pp = e.pp;
    a.n = e.n;
    a.ld = e.ld;
    a.n_pp = e.n_pp;
#pragma unroll
    for (int k = 0; k < kMaxPP; ++k) a.slot[k] = e.slot[k];
    a.p = tab.sp[e.sys];
    a.h = e.h;
    a.h2 = e.h2;
    a.h6 = e.h6;
    a.steps = tab.steps;
    a.ckpt = nullptr;
    a.ckpt_c = nullptr;
    a.ckpt_ld = 0;
    rk4_tile<SysT<R>, R, KAHAN, PPT>(a, (int64_t)(t - e.tile_begin) * blockDim.x * PPT);
}

template <typename R> using HH1 = HHRing<R, 1>;
template <typename R> using HH3 = HHRing<R, 3>;
template <typename R> using Lin1 = Linear<R, 1>;
template <typename R> using Lin2 = Linear<R, 2>;
template <typename R> using Lin3 = Linear<R, 3>;
template <typename R> using Lin4 = Linear<R, 4>;

template <typename R, bool KAHAN, int PPT>
__global__ void __launch_bounds__(256) k_groups(GroupTable tab, unsigned int* counter) {
    constexpr int PH = PPT > 2 ? 2 : PPT;  // the rings run at most 2 particles per thread
    __shared__ int s_t;
    for (;;) {
        if (threadIdx.x == 0) s_t = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int t = s_t;
        __syncthreads();
        if (t >= tab.ntiles) return;
        int g = 0;
        while (g + 1 < tab.ngroups && tab.g[g + 1].tile_begin <= t) ++g;
        const GroupEntry& e = tab.g[g];
        switch (e.kind) {
            case K_LORENZ: run_tile<Lorenz, R, KAHAN, PPT>(tab, e, t); break;
            case K_WC: run_tile<WilsonCowan, R, KAHAN, PPT>(tab, e, t); break;
            case K_HH1: run_tile<HH1, R, KAHAN, PH>(tab, e, t); break;
            case K_HH3: run_tile<HH3, R, KAHAN, PH>(tab, e, t); break;
            case K_LIN1: run_tile<Lin1, R, KAHAN, PPT>(tab, e, t); break;
            case K_LIN2: run_tile<Lin2, R, KAHAN, PPT>(tab, e, t); break;
            case K_LIN3: run_tile<Lin3, R, KAHAN, PPT>(tab, e, t); break;
            case K_LIN4: run_tile<Lin4, R, KAHAN, PPT>(tab, e, t); break;
        }
    }
}

__global__ void k_reset_counter(unsigned int* c) { *c = 0u; }

int kind_of(const ff_system_s* s) {
    switch (s->rhs) {
        case FF_RHS_LORENZ: return K_LORENZ;
        case FF_RHS_WILSON_COWAN: return K_WC;
        case FF_RHS_HH_RING: return s->dim == 5 ? K_HH1 : K_HH3;
        case FF_RHS_LINEAR: return K_LIN1 + s->dim - 1;
    }
    return -1;
}

// Relative cost of one particle-step, for ordering tiles (dearest first).
double cost_of(int kind) {
    switch (kind) {
        case K_HH3: return 30.0;
        case K_HH1: return 10.0;
        case K_WC: return 3.0;
        default: return 1.0;
    }
}

int ppt_of(int kind, int ppt) { return (kind == K_HH1 || kind == K_HH3) ? std::min(ppt, 2) : ppt; }

template <typename R, bool KAHAN>
hipError_t launch_groups_t(const GroupTable& tab, int ppt, int block, unsigned int* counter, hipStream_t st,
                           int cus) {
    auto go = [&](auto kern) -> hipError_t {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, 0);
        if (e != hipSuccess || per_cu < 1) per_cu = 1;
        const int grid = std::max(1, std::min(tab.ntiles, per_cu * cus));
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, counter);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, tab, counter);
        return hipGetLastError();
    };
    switch (ppt) {
        case 4: return go(k_groups<R, KAHAN, 4>);
        case 2: return go(k_groups<R, KAHAN, 2>);
        default: return go(k_groups<R, KAHAN, 1>);
    }
}

hipError_t launch_groups(int prec, const GroupTable& tab, int ppt, int block, unsigned int* counter,
                         hipStream_t st, int cus) {
    switch (prec) {
        case FF_FP64: return launch_groups_t<double, false>(tab, ppt, block, counter, st, cus);
        case FF_FP32: return launch_groups_t<float, false>(tab, ppt, block, counter, st, cus);
        case FF_FP32_KAHAN: return launch_groups_t<float, true>(tab, ppt, block, counter, st, cus);
    }
    return hipErrorInvalidValue;
}

std::mutex g_mu;
std::vector<unsigned int*> g_counter;  // library-owned counters, one per device
std::vector<int> g_cus;

ff_status device_info(unsigned int** counter, int* cus, bool need_counter, hipStream_t st) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_cus.size() <= dev) {
        g_cus.resize(dev + 1, 0);
        g_counter.resize(dev + 1, nullptr);
    }
    if (!g_cus[dev]) {
        int c = 0;
        e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return device_fail(e, "hipDeviceGetAttribute");
        g_cus[dev] = c;
    }
    *cus = g_cus[dev];
    if (need_counter && !g_counter[dev]) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
            return fail(FF_E_NOMEM, "pass `workspace` to ff_integrate_groups under stream capture");
        e = hipMalloc(&g_counter[dev], 256);
        if (e != hipSuccess) return fail(FF_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    if (need_counter) *counter = g_counter[dev];
    return FF_OK;
}

struct Prepared {
    std::vector<GroupTable> tables;
    int prec = -1;
};

ff_status prepare(const ff_group* groups, int32_t n_groups, const ff_tuning& t, Prepared* out) {
    if (!groups && n_groups > 0) return fail(FF_E_INVALID, "groups is NULL");
    if (n_groups < 0) return fail(FF_E_INVALID, "n_groups < 0");
    struct Item {
        int idx, kind;
        double cost;
    };
    std::vector<Item> items;
    for (int i = 0; i < n_groups; ++i) {
        const ff_group& g = groups[i];
        if (ff_status s = check_system(g.sys)) return s;
        if (g.sys->expr)
            return fail(FF_E_UNSUPPORTED, "the ragged-batch kernel holds the built-in right-hand sides only");
        if (ff_status s = check_batch(g.sys, &g.b, true)) return s;
        if (!std::isfinite(g.dt_signed)) return fail(FF_E_INVALID, "group dt_signed is not finite");
        if (g.b.n > 0x7fffffffLL) return fail(FF_E_UNSUPPORTED, "group larger than 2^31 - 1 particles");
        if (out->prec < 0) out->prec = g.b.prec;
        if (g.b.prec != out->prec) return fail(FF_E_INVALID, "all groups of one call must have the same precision");
        if (g.b.n == 0 || g.dt_signed == 0.0) continue;
        const int k = kind_of(g.sys);
        items.push_back({i, k, cost_of(k)});
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
    GroupTable tab;
    std::memset(&tab, 0, sizeof tab);
    std::vector<const ff_system_s*> sysv;
    auto flush = [&]() {
        if (tab.ngroups > 0) out->tables.push_back(tab);
        std::memset(&tab, 0, sizeof tab);
        sysv.clear();
    };
    for (const Item& it : items) {
        const ff_group& g = groups[it.idx];
        int si = -1;
        for (int k = 0; k < (int)sysv.size(); ++k)
            if (sysv[k] == g.sys) si = k;
        if (tab.ngroups == kMaxGroups || (si < 0 && (int)sysv.size() == kMaxSys)) {
            flush();
            si = -1;
        }
        if (si < 0) {
            si = (int)sysv.size();
            sysv.push_back(g.sys);
            for (int q = 0; q < kMaxParams; ++q) tab.sp[si].v[q] = q < g.sys->n_params ? g.sys->params[q] : 0.0;
        }
        const RK4Launch L = make_launch(g.sys, &g.b, g.dt_signed, &t, nullptr);
        GroupEntry& e = tab.g[tab.ngroups];
        e.state = g.b.state;
        e.comp = g.b.comp;
        e.pp = g.b.pparams;
        e.ld = g.b.ld;
        e.n = (int32_t)g.b.n;
        e.kind = (int8_t)it.kind;
        e.sys = (int8_t)si;
        e.n_pp = (int8_t)g.b.n_pp;
        e.ppt = (int8_t)ppt_of(it.kind, t.particles_per_thread);
        for (int k = 0; k < kMaxPP; ++k) e.slot[k] = (int8_t)L.slot[k];
        e.h = L.h;
        e.h2 = L.h2;
        e.h6 = L.h6;
        const int64_t per_tile = (int64_t)t.block * e.ppt;
        const int64_t tiles = (g.b.n + per_tile - 1) / per_tile;
        if ((int64_t)tab.ntiles + tiles > 0x7fffffffLL) return fail(FF_E_UNSUPPORTED, "too many tiles");
        e.tile_begin = tab.ntiles;
        tab.ntiles += (int32_t)tiles;
        ++tab.ngroups;
    }
    flush();
    return FF_OK;
}

ff_status run_prepared(Prepared& P, int64_t nsteps, const ff_tuning& t, unsigned int* counter, int cus,
                       hipStream_t st) {
    for (GroupTable& tab : P.tables) {
        for (int64_t done = 0; done < nsteps;) {
            tab.steps = std::min<int64_t>(t.steps_per_launch, nsteps - done);
            const hipError_t e = launch_groups(P.prec, tab, t.particles_per_thread, t.block, counter, st, cus);
            if (e != hipSuccess) return device_fail(e, "ff_integrate_groups launch");
            done += tab.steps;
        }
    }
    return FF_OK;
}

// Autotune choices per group list.  When the environment variable
// FF_AUTOTUNE_CACHE names a file, its lines "<signature> <steps_per_launch>
// <particles_per_thread> <block>" are read at the first lookup of the process
// (malformed lines are skipped) and every new choice is appended to it.  The
// file only saves tuning time: a write that fails is ignored.
std::mutex g_tune_mu;
std::map<std::string, ff_tuning> g_tune_cache;
bool g_tune_file_read = false;

const char* tune_file() {
    const char* p = std::getenv("FF_AUTOTUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

bool valid_tuning(long long s, int ppt, int block) {
    return s >= 1 && s <= 0x7fffffffLL && (ppt == 1 || ppt == 2 || ppt == 4) && block >= 64 && block <= 256 &&
           block % 64 == 0;
}

// Caller holds g_tune_mu.
void read_tune_file() {
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char* path = tune_file();
    if (!path) return;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ss(line);
        std::string key;
        long long steps = 0;
        int ppt = 0, block = 0;
        if (!(ss >> key >> steps >> ppt >> block) || !valid_tuning(steps, ppt, block)) continue;
        g_tune_cache[key] = ff_tuning{(int32_t)steps, ppt, block};
    }
}

// Caller holds g_tune_mu.
bool find_tuning(const std::string& key, ff_tuning* t) {
    read_tune_file();
    auto it = g_tune_cache.find(key);
    if (it == g_tune_cache.end()) return false;
    *t = it->second;
    return true;
}

// Caller holds g_tune_mu.
void store_tuning(const std::string& key, const ff_tuning& t) {
    g_tune_cache[key] = t;
    if (const char* path = tune_file()) {
        std::ofstream out(path, std::ios::app);
        out << key << ' ' << t.steps_per_launch << ' ' << t.particles_per_thread << ' ' << t.block << '\n';
    }
}

std::string signature(const ff_group* groups, int32_t n_groups, int64_t nsteps) {
    std::string s = std::to_string(nsteps);
    for (int i = 0; i < n_groups; ++i) {
        const ff_group& g = groups[i];
        s += "|" + std::to_string(g.sys->rhs) + "," + std::to_string(g.sys->dim) + "," + std::to_string(g.b.prec) +
             "," + std::to_string(g.b.n) + "," + std::to_string(g.b.n_pp);
    }
    return s;
}

}  // namespace

}  // namespace ff

using namespace ff;

extern "C" {

ff_status ff_groups_workspace_size(int32_t n_groups, size_t* bytes) {
    set_error("");
    if (!bytes) return fail(FF_E_INVALID, "bytes is NULL");
    if (n_groups < 0) return fail(FF_E_INVALID, "n_groups < 0");
    *bytes = 256;
    return FF_OK;
}

ff_status ff_integrate_groups(const ff_group* groups, int32_t n_groups, int64_t nsteps, const ff_tuning* tuning,
                              void* workspace, size_t workspace_bytes, void* stream) {
    set_error("");
    if (nsteps < 0) return fail(FF_E_INVALID, "nsteps < 0");
    ff_tuning t;
    if (tuning) {
        if (ff_status s = check_tuning(nullptr, tuning)) return s;
        t = *tuning;
    } else {
        t.steps_per_launch = (int32_t)std::min<int64_t>(std::max<int64_t>(nsteps, 1), 4096);
        t.particles_per_thread = 1;
        t.block = 256;
    }
    Prepared P;
    if (ff_status s = prepare(groups, n_groups, t, &P)) return s;
    if (!tuning) {
        // the groups are valid now: take ff_autotune's choice for this list
        bool hit = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            hit = find_tuning(signature(groups, n_groups, nsteps), &t);
        }
        if (hit) {
            P = Prepared();
            if (ff_status s = prepare(groups, n_groups, t, &P)) return s;
        }
    }
    if (nsteps == 0 || P.tables.empty()) return FF_OK;
    if (workspace && workspace_bytes < 256) return fail(FF_E_NOMEM, "groups workspace needs 256 bytes");
    hipStream_t st = (hipStream_t)stream;
    unsigned int* counter = (unsigned int*)workspace;
    int cus = 0;
    if (ff_status s = device_info(&counter, &cus, workspace == nullptr, st)) return s;
    if (workspace) counter = (unsigned int*)workspace;
    return run_prepared(P, nsteps, t, counter, cus, st);
}

ff_status ff_autotune(const ff_group* groups, int32_t n_groups, int64_t nsteps, ff_tuning* out, void* stream) {
    set_error("");
    if (!out) return fail(FF_E_INVALID, "out is NULL");
    if (nsteps < 1) return fail(FF_E_INVALID, "nsteps < 1");
    ff_tuning probe{1, 1, 256};
    {
        Prepared P;
        if (ff_status s = prepare(groups, n_groups, probe, &P)) return s;
        if (P.tables.empty()) {
            *out = ff_tuning{(int32_t)std::min<int64_t>(nsteps, 500), 1, 256};
            return FF_OK;
        }
    }
    const std::string key = signature(groups, n_groups, nsteps);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (find_tuning(key, out)) return FF_OK;
    }
    hipStream_t st = (hipStream_t)stream;
    unsigned int* counter = nullptr;
    int cus = 0;
    if (ff_status s = device_info(&counter, &cus, true, st)) return s;
    // work on copies so the caller's state is untouched
    std::vector<ff_group> copy(groups, groups + n_groups);
    std::vector<void*> owned;
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        for (void* p : owned) (void)hipFree(p);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    for (ff_group& g : copy) {
        if (g.b.n == 0) continue;
        // the slice's rows d*ld + [0, n) from its first particle: the span ends
        // n elements into the last row, inside the caller's [dim][ld] array
        const size_t bytes = ((size_t)(g.sys->dim - 1) * g.b.ld + g.b.n) * prec_size(g.b.prec);
        for (void** field : {&g.b.state, &g.b.comp}) {
            if (!*field) continue;
            void* p = nullptr;
            if (hipMalloc(&p, bytes) != hipSuccess) {
                cleanup();
                return fail(FF_E_NOMEM, "ff_autotune: hipMalloc of a state copy failed");
            }
            owned.push_back(p);
            if (hipError_t e = hipMemcpyAsync(p, *field, bytes, hipMemcpyDeviceToDevice, st)) {
                cleanup();
                return device_fail(e, "ff_autotune: copy of the state");
            }
            *field = p;
        }
    }
    for (hipEvent_t& e : ev) {
        if (hipError_t err = hipEventCreate(&e)) {
            e = nullptr;
            cleanup();
            return device_fail(err, "ff_autotune: hipEventCreate");
        }
    }
    const int64_t tune_steps = std::min<int64_t>(nsteps, 200);
    // one candidate: a warm-up, then one timed run of tune_steps steps
    auto trial = [&](const ff_tuning& t, float* ms) -> ff_status {
        Prepared P;
        if (ff_status s = prepare(copy.data(), n_groups, t, &P)) return s;
        if (ff_status s = run_prepared(P, std::min<int64_t>(t.steps_per_launch, tune_steps), t, counter, cus, st))
            return s;
        if (hipError_t e = hipEventRecord(ev[0], st)) return device_fail(e, "ff_autotune: hipEventRecord");
        if (ff_status s = run_prepared(P, tune_steps, t, counter, cus, st)) return s;
        if (hipError_t e = hipEventRecord(ev[1], st)) return device_fail(e, "ff_autotune: hipEventRecord");
        if (hipError_t e = hipEventSynchronize(ev[1])) return device_fail(e, "ff_autotune: hipEventSynchronize");
        if (hipError_t e = hipEventElapsedTime(ms, ev[0], ev[1]))
            return device_fail(e, "ff_autotune: hipEventElapsedTime");
        return FF_OK;
    };
    float best = 1e30f;
    ff_tuning bestt{(int32_t)std::min<int64_t>(nsteps, 500), 1, 256};
    const int64_t smax = std::min<int64_t>(500, nsteps);
    std::vector<int64_t> svals;
    for (int64_t s : {10, 20, 50, 100, 200, 500})
        if (s <= smax) svals.push_back(s);
    if (svals.empty() || svals.back() != smax) svals.push_back(smax);
    for (int ppt : {1, 2, 4}) {
        for (int block : {128, 256}) {
            for (int64_t s : svals) {
                const ff_tuning t{(int32_t)s, ppt, block};
                float ms = 0.f;
                if (ff_status status = trial(t, &ms)) {
                    cleanup();
                    return status;
                }
                if (ms < best) {
                    best = ms;
                    bestt = t;
                }
            }
        }
    }
    cleanup();
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        store_tuning(key, bestt);
    }
    *out = bestt;
    return FF_OK;
}

}  // extern "C"
