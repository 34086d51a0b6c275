// C-ABI of libsem.so, batch side: mixed-order batch plans (tile tables,
// autotuner, JSON plan cache) and the SSP-RK3 step captured in a HIP graph.
// The operations themselves are documented in include/sem.h; the kernels
// live in batch_*.hip and kernels_*.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sem.h"
#include "sem_cache.hpp"
#include "sem_host.hpp"
#include "sem_internal.hpp"

using namespace semapi;

namespace {

struct OrderChoice {
    int nq = 0;
    int epb = 0;
    int lay = semk::FULL;
    double us = -1.0;        // measured time of this order alone (autotuned), else -1
    int64_t elements = 0;
};

struct PlanCore {
    sem_dtype dtype = SEM_F64;
    semk::Phys phys{};
    int nt = 256;
    int lds_bytes = 0;
    int ntiles = 0;
    int device = 0;
    bool rk = false;                    // fused Runge-Kutta stage epilogue
    semk::RkStage rk_stage{0.0, 0.0, 0.0};
    std::vector<sem_block> blocks;
    std::vector<const void*> rk_x;      // per block, fused stage only
    std::vector<OrderChoice> orders;    // one per distinct Nq
    semh::Tile* d_tiles = nullptr;
    void* d_blocks = nullptr;
    bool autotuned = false;
    bool from_cache = false;
};

void free_core(PlanCore* p)
{
    if (!p)
        return;
    if (p->d_tiles)
        (void)hipFree(p->d_tiles);
    if (p->d_blocks)
        (void)hipFree(p->d_blocks);
    p->d_tiles = nullptr;
    p->d_blocks = nullptr;
}

sem_status check_block(const sem_block& b, int idx, sem_dtype dt, const sem_phys* phys)
{
    sem_status st = check_volume_args(b.Ne, b.Nq, dt, b.D, b.geo, b.q, b.rho_ref, b.theta_ref, phys,
                                      b.rhs);
    if (st != SEM_OK) {
        std::string m = last_error();
        return fail(st, "block %d: %s", idx, m.c_str());
    }
    return SEM_OK;
}

template <typename T>
std::vector<semk::BatchBlock<T>> host_block_table(const PlanCore& p)
{
    std::vector<semk::BatchBlock<T>> v;
    v.reserve(p.blocks.size());
    for (size_t i = 0; i < p.blocks.size(); ++i) {
        const sem_block& b = p.blocks[i];
        semk::BlockPtrs<T> bp = block_ptrs<T>(b.Ne, b.D, b.geo, b.q, b.rho_ref, b.theta_ref, b.rhs);
        if (p.rk)
            bp.rk_x = static_cast<const T*>(p.rk_x[i]);
        v.push_back(semk::BatchBlock<T>{bp, p.phys, p.rk_stage});
    }
    return v;
}

const OrderChoice& choice_for(const std::vector<OrderChoice>& orders, int nq)
{
    for (const OrderChoice& o : orders)
        if (o.nq == nq)
            return o;
    return orders.front();   // unreachable: every block's order has a choice
}

// Tiles of every block whose order is in `only_nq` (all if 0), sorted by
// decreasing estimated cost (longest-processing-time first, stable).
std::vector<semh::Tile> make_tiles(const std::vector<sem_block>& blocks,
                                   const std::vector<OrderChoice>& orders, int only_nq)
{
    struct Item {
        semh::Tile t;
        double cost;
    };
    std::vector<Item> items;
    for (size_t bi = 0; bi < blocks.size(); ++bi) {
        const sem_block& b = blocks[bi];
        if (only_nq && b.Nq != only_nq)
            continue;
        const OrderChoice& oc = choice_for(orders, b.Nq);
        const int vid = semh::variant_index(b.Nq, oc.epb, oc.lay);
        const double nodes = (double)b.Nq * b.Nq * b.Nq;
        // measured per-element time when autotuned, else a node count
        const double per_elem = (oc.us > 0 && oc.elements > 0) ? oc.us / oc.elements : nodes;
        for (int64_t e0 = 0; e0 < b.Ne; e0 += oc.epb) {
            const int ne = (int)std::min<int64_t>(oc.epb, b.Ne - e0);
            items.push_back({semh::Tile{(int32_t)bi, vid, ne, 0, e0}, per_elem * oc.epb});
        }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const Item& a, const Item& b) { return a.cost > b.cost; });
    std::vector<semh::Tile> out;
    out.reserve(items.size());
    for (const Item& it : items)
        out.push_back(it.t);
    return out;
}

int shape_lds(sem_dtype dt, int nt, int nq, int epb, int lay)
{
    return dt == SEM_F64 ? semh::batch_lds_bytes<double>(nt, nq, epb, lay)
                         : semh::batch_lds_bytes<float>(nt, nq, epb, lay);
}

int lds_for(sem_dtype dt, int nt, const std::vector<OrderChoice>& orders)
{
    int lds = 0;
    for (const OrderChoice& o : orders)
        lds = std::max(lds, shape_lds(dt, nt, o.nq, o.epb, o.lay));
    return lds;
}

bool variant_ok(sem_dtype dt, int nt, int nq, int epb, int lay, bool rk)
{
    return dt == SEM_F64 ? semh::batch_variant_ok<double>(nt, nq, epb, lay, rk)
                         : semh::batch_variant_ok<float>(nt, nq, epb, lay, rk);
}

hipError_t occupancy(sem_dtype dt, int nt, int lds, bool rk, int* bpc)
{
    return dt == SEM_F64 ? semh::batch_blocks_per_cu<double>(nt, lds, rk, bpc)
                         : semh::batch_blocks_per_cu<float>(nt, lds, rk, bpc);
}

hipError_t launch(const PlanCore& p, const semh::Tile* d_tiles, int ntiles, int lds, hipStream_t s)
{
    if (p.dtype == SEM_F64)
        return semh::launch_batch<double>(p.nt, d_tiles, ntiles,
                                          static_cast<const semk::BatchBlock<double>*>(p.d_blocks),
                                          p.rk, lds, s);
    return semh::launch_batch<float>(p.nt, d_tiles, ntiles,
                                     static_cast<const semk::BatchBlock<float>*>(p.d_blocks), p.rk,
                                     lds, s);
}

// The batch kernel must fit at least one workgroup per CU with `lds` bytes.
sem_status check_resident(const PlanCore& p, int lds)
{
    int bpc = 0;
    hipError_t err = occupancy(p.dtype, p.nt, lds, p.rk, &bpc);
    if (err != hipSuccess)
        return hip_fail(err, "occupancy query");
    if (bpc < 1)
        return fail(SEM_ERR_UNSUPPORTED, "batch kernel cannot be resident with %d B of LDS", lds);
    return SEM_OK;
}

sem_status upload_blocks(PlanCore& p, hipStream_t s)
{
    if (p.d_blocks)
        (void)hipFree(p.d_blocks);
    p.d_blocks = nullptr;
    const size_t bt_bytes = p.blocks.size() *
                            (p.dtype == SEM_F64 ? sizeof(semk::BatchBlock<double>)
                                                : sizeof(semk::BatchBlock<float>));
    hipError_t err = hipMalloc(&p.d_blocks, bt_bytes);
    if (err != hipSuccess)
        return fail(SEM_ERR_NO_MEMORY, "plan block table (%zu B): %s", bt_bytes,
                    hipGetErrorString(err));
    if (p.dtype == SEM_F64) {
        auto hb = host_block_table<double>(p);
        err = hipMemcpyAsync(p.d_blocks, hb.data(), bt_bytes, hipMemcpyHostToDevice, s);
        if (err == hipSuccess)
            err = hipStreamSynchronize(s);
    } else {
        auto hb = host_block_table<float>(p);
        err = hipMemcpyAsync(p.d_blocks, hb.data(), bt_bytes, hipMemcpyHostToDevice, s);
        if (err == hipSuccess)
            err = hipStreamSynchronize(s);
    }
    if (err != hipSuccess)
        return hip_fail(err, "upload block table");
    return SEM_OK;
}

// Upload the tile table for the current choices and check that the chosen
// workgroup size and LDS can be resident.
sem_status finalize(PlanCore& p, hipStream_t s)
{
    SEM_TRY(upload_blocks(p, s));
    if (p.d_tiles)
        (void)hipFree(p.d_tiles);
    p.d_tiles = nullptr;
    std::vector<semh::Tile> tiles = make_tiles(p.blocks, p.orders, 0);
    p.ntiles = (int)tiles.size();
    p.lds_bytes = lds_for(p.dtype, p.nt, p.orders);
    hipError_t err = hipMalloc((void**)&p.d_tiles, tiles.size() * sizeof(semh::Tile));
    if (err != hipSuccess)
        return fail(SEM_ERR_NO_MEMORY, "plan tile table: %s", hipGetErrorString(err));
    err = hipMemcpyAsync(p.d_tiles, tiles.data(), tiles.size() * sizeof(semh::Tile),
                         hipMemcpyHostToDevice, s);
    if (err == hipSuccess)
        err = hipStreamSynchronize(s);
    if (err != hipSuccess)
        return hip_fail(err, "upload tile table");
    return check_resident(p, p.lds_bytes);
}

// ---------------------------------------------------------------------------
// Plan cache (file format in sem_cache.cpp): a flat JSON object in
// the file named by SEM_PLAN_CACHE, keyed by device arch, dtype, workgroup
// size, the LDS cap of the launch, Nq and a power-of-two element bucket.
// ---------------------------------------------------------------------------
std::mutex g_cache_mu;

std::string cache_path()
{
    const char* p = getenv("SEM_PLAN_CACHE");
    return p ? std::string(p) : std::string();
}

std::string arch_name(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

std::string cache_key(const std::string& arch, sem_dtype dt, bool rk, int nt, int cap, int nq,
                      int64_t ne)
{
    int64_t bucket = 1;
    while (bucket < ne)
        bucket <<= 1;
    char buf[160];
    snprintf(buf, sizeof buf, "%s/%s%s/nt%d/lds%d/nq%d/ne%lld", arch.c_str(),
             dt == SEM_F64 ? "f64" : "f32", rk ? "-rk" : "", nt, cap, nq, (long long)bucket);
    return buf;
}

// Time one order's blocks alone with the shape currently in p.orders, under
// the dynamic LDS `cap` that the combined launch will use (it sets the
// occupancy): median of 5 launches after 2 warm-ups, HIP events.
sem_status time_candidate(PlanCore& p, int nq, int cap, hipStream_t s, double* us_out)
{
    std::vector<semh::Tile> tiles = make_tiles(p.blocks, p.orders, nq);
    SEM_TRY(check_resident(p, cap));
    semh::Tile* d_t = nullptr;
    hipError_t err = hipMalloc((void**)&d_t, tiles.size() * sizeof(semh::Tile));
    if (err != hipSuccess)
        return fail(SEM_ERR_NO_MEMORY, "autotune tile table: %s", hipGetErrorString(err));
    err = hipMemcpy(d_t, tiles.data(), tiles.size() * sizeof(semh::Tile), hipMemcpyHostToDevice);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (err == hipSuccess)
        err = hipEventCreate(&e0);
    if (err == hipSuccess)
        err = hipEventCreate(&e1);
    std::vector<float> ms;
    for (int r = 0; r < 7 && err == hipSuccess; ++r) {
        err = hipEventRecord(e0, s);
        if (err == hipSuccess)
            err = launch(p, d_t, (int)tiles.size(), cap, s);
        if (err == hipSuccess)
            err = hipEventRecord(e1, s);
        if (err == hipSuccess)
            err = hipEventSynchronize(e1);
        float t = 0.f;
        if (err == hipSuccess && r >= 2 && hipEventElapsedTime(&t, e0, e1) == hipSuccess)
            ms.push_back(t);
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(d_t);
    if (err != hipSuccess)
        return hip_fail(err, "autotune launch");
    std::sort(ms.begin(), ms.end());
    *us_out = ms.empty() ? 1e30 : 1e3 * ms[ms.size() / 2];
    return SEM_OK;
}

constexpr std::chrono::milliseconds kSettle{30};

// For every workgroup size and every LDS cap (the LDS of a compiled shape),
// pick per order the fastest shape that fits under the cap, timed at that
// cap; keep the (size, cap) whose per-order times sum lowest.  The launch's
// occupancy is set by its largest shape, so timing each order at the cap it
// will share is what makes the per-order choices add up.
sem_status autotune(PlanCore& p, bool use_cache, hipStream_t s)
{
    const std::string arch = arch_name(p.device);
    const std::string path = use_cache ? cache_path() : std::string();
    std::map<std::string, semcache::Entry> cache;
    if (!path.empty()) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        cache = semcache::read(path);
    }
    SEM_TRY(upload_blocks(p, s));
    bool all_cached = true;
    bool settled = false;
    double best_total = 1e300;
    int best_nt = 0, best_cap = 0;
    std::vector<OrderChoice> best_orders;
    for (int nt : semh::kBatchThreads) {
        p.nt = nt;
        std::vector<int> caps;
        for (int i = 0; i < semh::kNumVariants; ++i) {
            const semh::VariantDef v = semh::kVariants[i];
            bool used = false;
            for (const OrderChoice& o : p.orders)
                used |= o.nq == v.nq;
            if (used && variant_ok(p.dtype, nt, v.nq, v.epb, v.lay, p.rk))
                caps.push_back(shape_lds(p.dtype, nt, v.nq, v.epb, v.lay));
        }
        std::sort(caps.begin(), caps.end());
        caps.erase(std::unique(caps.begin(), caps.end()), caps.end());
        for (int cap : caps) {
            std::vector<OrderChoice> chosen = p.orders;
            double total = 0.0;
            bool feasible = true;
            for (OrderChoice& oc : chosen) {
                const std::string key = cache_key(arch, p.dtype, p.rk, nt, cap, oc.nq, oc.elements);
                auto it = cache.find(key);
                if (it != cache.end() &&
                    variant_ok(p.dtype, nt, oc.nq, it->second.epb, it->second.lay, p.rk) &&
                    shape_lds(p.dtype, nt, oc.nq, it->second.epb, it->second.lay) <= cap) {
                    oc.epb = it->second.epb;
                    oc.lay = it->second.lay;
                    oc.us = it->second.us;
                    total += oc.us;
                    continue;
                }
                double best = 1e300;
                int best_epb = -1, best_lay = 0;
                for (int i = 0; i < semh::kNumVariants; ++i) {
                    const semh::VariantDef v = semh::kVariants[i];
                    if (v.nq != oc.nq || !variant_ok(p.dtype, nt, v.nq, v.epb, v.lay, p.rk) ||
                        shape_lds(p.dtype, nt, v.nq, v.epb, v.lay) > cap)
                        continue;
                    all_cached = false;
                    for (OrderChoice& o : p.orders)
                        if (o.nq == oc.nq) {
                            o.epb = v.epb;
                            o.lay = v.lay;
                        }
                    double us = 0.0;
                    if (!settled) {
                        // the shader clock ramps up over the first milliseconds
                        // of load; keep launching before the first timing so
                        // that no candidate is timed on the ramp
                        const auto t0 = std::chrono::steady_clock::now();
                        do
                            SEM_TRY(time_candidate(p, oc.nq, cap, s, &us));
                        while (std::chrono::steady_clock::now() - t0 < kSettle);
                        settled = true;
                    }
                    SEM_TRY(time_candidate(p, oc.nq, cap, s, &us));
                    if (log_enabled())
                        fprintf(stderr, "[semvol] autotune %s nt=%d lds<=%d nq=%d epb=%d layout=%d: %.2f us\n",
                                p.dtype == SEM_F64 ? "f64" : "f32", nt, cap, v.nq, v.epb, v.lay, us);
                    if (us < best) {
                        best = us;
                        best_epb = v.epb;
                        best_lay = v.lay;
                    }
                }
                if (best_epb < 0) {
                    feasible = false;
                    break;
                }
                oc.epb = best_epb;
                oc.lay = best_lay;
                oc.us = best;
                total += best;
                cache[key] = semcache::Entry{best_epb, best_lay, best};
            }
            if (feasible && total < best_total) {
                best_total = total;
                best_nt = nt;
                best_cap = cap;
                best_orders = chosen;
            }
        }
    }
    if (best_orders.empty())
        return fail(SEM_ERR_UNSUPPORTED, "no batch tile shape fits every order of the plan");
    p.nt = best_nt;
    p.orders = best_orders;
    p.autotuned = true;
    p.from_cache = all_cached;
    if (!path.empty() && !all_cached) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto merged = semcache::read(path);
        for (auto& kv : cache)
            merged[kv.first] = kv.second;
        semcache::write(path, merged);
    }
    if (log_enabled())
        fprintf(stderr, "[semvol] autotune chose nt=%d, LDS cap %d B (sum of per-order times %.2f us)%s\n",
                p.nt, best_cap, best_total, all_cached ? " from cache" : "");
    return SEM_OK;
}

// The built-in shape of one order in a launch of nt threads: the
// single-order default tile, else the historical small shape with all fluxes
// resident, else the same count aliased.  False if none fits.
bool default_shape(sem_dtype dt, int nt, int nq, bool rk, int* epb, int* lay)
{
    const DefaultTile dft = default_tile(dt, nq);
    if (variant_ok(dt, nt, nq, dft.epb, dft.lay, rk)) {
        *epb = dft.epb;
        *lay = dft.lay;
        return true;
    }
    *epb = default_epb(nq);
    for (int l : {(int)semk::FULL, (int)semk::ALIAS})
        if (variant_ok(dt, nt, nq, *epb, l, rk)) {
            *lay = l;
            return true;
        }
    return false;
}

// Built-in batch shapes (no autotuning): the smallest workgroup size among
// 256, 512 and 1024 for which every order has a built-in shape.
sem_status default_shapes(PlanCore& p)
{
    for (int nt : semh::kBatchThreads) {
        bool all = true;
        for (OrderChoice& o : p.orders)
            all = all && default_shape(p.dtype, nt, o.nq, p.rk, &o.epb, &o.lay);
        if (all) {
            p.nt = nt;
            return SEM_OK;
        }
    }
    return fail(SEM_ERR_UNSUPPORTED, "no default batch shape covers every order of the plan");
}

}  // namespace

bool semapi::batch_default_shape(sem_dtype dt, int nt, int nq, int* epb, int* lay)
{
    return default_shape(dt, nt, nq, false, epb, lay);
}

namespace {

sem_status build_plan(const sem_block* blocks, int32_t nblocks, sem_dtype dt, const sem_phys* phys,
                      uint32_t flags, hipStream_t s, const PlanCore* template_plan,
                      const semk::RkStage* rk, const void* const* rk_x, PlanCore** out)
{
    SEM_TRY(check_dtype(dt));
    if (!out)
        return fail(SEM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!blocks || nblocks < 1)
        return fail(SEM_ERR_INVALID_ARG, "need at least one block (nblocks = %d)", nblocks);
    if (!phys)
        return fail(SEM_ERR_INVALID_ARG, "phys is NULL");
    for (int i = 0; i < nblocks; ++i)
        SEM_TRY(check_block(blocks[i], i, dt, phys));
    PlanCore* p = new (std::nothrow) PlanCore();
    if (!p)
        return fail(SEM_ERR_NO_MEMORY, "plan allocation");
    p->dtype = dt;
    p->phys = to_phys(phys);
    p->blocks.assign(blocks, blocks + nblocks);
    if (rk) {
        p->rk = true;
        p->rk_stage = *rk;
        p->rk_x.assign(rk_x, rk_x + nblocks);
    }
    hipError_t err = hipGetDevice(&p->device);
    if (err == hipSuccess)
        err = dt == SEM_F64 ? semh::batch_prepare<double>() : semh::batch_prepare<float>();
    if (err != hipSuccess) {
        delete p;
        return hip_fail(err, "batch kernel setup");
    }
    for (int i = 0; i < nblocks; ++i) {
        bool found = false;
        for (OrderChoice& o : p->orders)
            if (o.nq == blocks[i].Nq) {
                o.elements += blocks[i].Ne;
                found = true;
            }
        if (!found) {
            OrderChoice o;
            o.nq = blocks[i].Nq;
            o.elements = blocks[i].Ne;
            p->orders.push_back(o);
        }
    }
    std::sort(p->orders.begin(), p->orders.end(),
              [](const OrderChoice& a, const OrderChoice& b) { return a.nq < b.nq; });
    sem_status st = SEM_OK;
    if (template_plan) {
        p->nt = template_plan->nt;
        p->orders = template_plan->orders;
        p->autotuned = template_plan->autotuned;
        p->from_cache = template_plan->from_cache;
    } else if (flags & SEM_PLAN_AUTOTUNE) {
        st = autotune(*p, (flags & SEM_PLAN_USE_CACHE) != 0, s);
    } else {
        st = default_shapes(*p);
    }
    if (st == SEM_OK)
        st = finalize(*p, s);
    if (st != SEM_OK) {
        free_core(p);
        delete p;
        return st;
    }
    *out = p;
    return SEM_OK;
}

}  // namespace

struct sem_plan_s {
    PlanCore core;
};

extern "C" sem_status sem_batch_plan(const sem_block* blocks, int32_t nblocks, sem_dtype dtype,
                                     const sem_phys* phys, uint32_t flags, void* stream,
                                     sem_plan* out)
{
    if (!out)
        return fail(SEM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    PlanCore* core = nullptr;
    SEM_TRY(build_plan(blocks, nblocks, dtype, phys, flags, static_cast<hipStream_t>(stream), nullptr,
                       nullptr, nullptr, &core));
    sem_plan p = new (std::nothrow) sem_plan_s();
    if (!p) {
        free_core(core);
        delete core;
        return fail(SEM_ERR_NO_MEMORY, "plan allocation");
    }
    p->core = *core;   // takes over the device tables
    delete core;
    *out = p;
    return SEM_OK;
}

extern "C" sem_status sem_batch_execute(sem_plan plan, void* stream)
{
    if (!plan)
        return fail(SEM_ERR_INVALID_ARG, "plan is NULL");
    const PlanCore& c = plan->core;
    if (!c.d_tiles || !c.d_blocks)
        return fail(SEM_ERR_INVALID_ARG, "plan has no device tables (destroyed?)");
    hipError_t err = launch(c, c.d_tiles, c.ntiles, c.lds_bytes, static_cast<hipStream_t>(stream));
    if (err != hipSuccess)
        return hip_fail(err, "batch kernel launch");
    return SEM_OK;
}

namespace {
std::string describe(const PlanCore& c)
{
    std::string s = "{\"dtype\": \"";
    s += c.dtype == SEM_F64 ? "f64" : "f32";
    char tmp[256];
    snprintf(tmp, sizeof tmp,
             "\", \"threads\": %d, \"lds_bytes\": %d, \"tiles\": %d, "
             "\"blocks\": %zu, \"fused_rk_stage\": %s, \"autotuned\": %s, \"from_cache\": %s, "
             "\"orders\": [",
             c.nt, c.lds_bytes, c.ntiles, c.blocks.size(), c.rk ? "true" : "false",
             c.autotuned ? "true" : "false", c.from_cache ? "true" : "false");
    s += tmp;
    for (size_t i = 0; i < c.orders.size(); ++i) {
        snprintf(tmp, sizeof tmp,
                 "%s{\"Nq\": %d, \"elems_per_block\": %d, \"layout\": \"%s\", \"elements\": %lld, "
                 "\"tuned_us\": %.3f}",
                 i ? ", " : "", c.orders[i].nq, c.orders[i].epb,
                 c.orders[i].lay == semk::ALIAS ? "alias" : "full", (long long)c.orders[i].elements,
                 c.orders[i].us);
        s += tmp;
    }
    s += "]}";
    return s;
}
}  // namespace

extern "C" sem_status sem_plan_describe(sem_plan plan, char* buf, int32_t len)
{
    if (!plan || !buf || len < 1)
        return fail(SEM_ERR_INVALID_ARG, "NULL plan or buffer");
    snprintf(buf, (size_t)len, "%s", describe(plan->core).c_str());
    return SEM_OK;
}

extern "C" sem_status sem_plan_destroy(sem_plan plan)
{
    if (!plan)
        return fail(SEM_ERR_INVALID_ARG, "plan is NULL");
    free_core(&plan->core);
    delete plan;
    return SEM_OK;
}

// ===========================================================================
// SSP-RK3 step in a HIP graph
// ===========================================================================
struct sem_rk3_s {
    PlanCore stage[3];
    bool fused = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" sem_status sem_rk3_graph_create(const sem_block* blocks, int32_t nblocks, sem_dtype dtype,
                                           const sem_phys* phys, uint32_t flags, void* q_n,
                                           void* q_1, void* q_2, void* L, int64_t n, double dt,
                                           void* stream, sem_rk3* out)
{
    if (!out)
        return fail(SEM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    SEM_TRY(check_dtype(dtype));
    const size_t es = elem_size(dtype);
    SEM_TRY(check_ptr(q_n, es, "q_n"));
    SEM_TRY(check_ptr(q_1, es, "q_1"));
    SEM_TRY(check_ptr(q_2, es, "q_2"));
    SEM_TRY(check_ptr(L, es, "L"));
    if (n < 1)
        return fail(SEM_ERR_INVALID_ARG, "n = %lld < 1", (long long)n);
    if (!blocks || nblocks < 1)
        return fail(SEM_ERR_INVALID_ARG, "need at least one block");
    if (!std::isfinite(dt))
        return fail(SEM_ERR_INVALID_ARG, "dt is not finite");
    const bool fused = (flags & SEM_RK3_SEPARATE_STAGES) == 0;
    // Shu-Osher coefficients: stage k writes a_k q_n + b_k (q_k + dt v(q_k))
    const double a[3] = {0.0, 0.75, 1.0 / 3.0};
    const double b[3] = {1.0, 0.25, 2.0 / 3.0};
    char* qin[3] = {static_cast<char*>(q_n), static_cast<char*>(q_1), static_cast<char*>(q_2)};
    char* qout[3] = {static_cast<char*>(q_1), static_cast<char*>(q_2), static_cast<char*>(q_n)};
    // every block's q inside q_n and its rhs inside L at the same offset
    std::vector<sem_block> sb[3];
    std::vector<const void*> xs(nblocks);
    const char* qn = static_cast<const char*>(q_n);
    const char* lb = static_cast<const char*>(L);
    for (int k = 0; k < 3; ++k)
        sb[k].assign(blocks, blocks + nblocks);
    {
        // the four buffers are distinct: each stage reads one and writes another
        const size_t nb = (size_t)n * es;
        const ByteRange bufs[] = {{"q_n", q_n, nb}, {"q_1", q_1, nb}, {"q_2", q_2, nb}, {"L", L, nb}};
        for (int i = 0; i < 4; ++i)
            SEM_TRY(check_output_overlap(bufs[i].name, bufs[i].p, nb, bufs + i + 1, 3 - i));
    }
    // the blocks' q arrays tile q_n[0, n) exactly, so that both stage modes
    // advance every value of q_n (and no value twice)
    {
        std::vector<std::pair<int64_t, int64_t>> spans;   // byte offset, length
        for (int i = 0; i < nblocks; ++i) {
            if (blocks[i].Ne < 1 || blocks[i].Nq < kMinNq || blocks[i].Nq > kMaxNq)
                return fail(SEM_ERR_INVALID_ARG, "block %d: Ne = %d, Nq = %d", i, blocks[i].Ne,
                            blocks[i].Nq);
            const int64_t m = (int64_t)blocks[i].Nq * blocks[i].Nq * blocks[i].Nq;
            spans.emplace_back(static_cast<const char*>(blocks[i].q) - static_cast<const char*>(q_n),
                               (int64_t)blocks[i].Ne * 5 * m * (int64_t)es);
        }
        std::sort(spans.begin(), spans.end());
        int64_t end = 0;
        for (const auto& sp : spans) {
            if (sp.first != end)
                return fail(SEM_ERR_INVALID_ARG,
                            "the blocks' q arrays must tile q_n[0, n) exactly: %s at byte %lld "
                            "(expected a block starting at byte %lld)",
                            sp.first < end ? "overlap" : "gap", (long long)sp.first, (long long)end);
            end += sp.second;
        }
        if (end != n * (int64_t)es)
            return fail(SEM_ERR_INVALID_ARG,
                        "the blocks' q arrays cover %lld of the %lld bytes of q_n[0, n)",
                        (long long)end, (long long)(n * (int64_t)es));
    }
    for (int i = 0; i < nblocks; ++i) {
        const int64_t m = (int64_t)blocks[i].Nq * blocks[i].Nq * blocks[i].Nq;
        const int64_t bytes = (int64_t)blocks[i].Ne * 5 * m * (int64_t)es;
        const int64_t off = static_cast<const char*>(blocks[i].q) - qn;
        const int64_t roff = static_cast<const char*>((const void*)blocks[i].rhs) - lb;
        if (off < 0 || off + bytes > n * (int64_t)es)
            return fail(SEM_ERR_INVALID_ARG, "block %d: q is not inside q_n[0, n)", i);
        if (roff != off)
            return fail(SEM_ERR_INVALID_ARG, "block %d: rhs is not at the same offset in L as q in q_n",
                        i);
        xs[i] = qn + off;
        for (int k = 0; k < 3; ++k) {
            sb[k][i].q = qin[k] + off;
            if (fused)
                sb[k][i].rhs = qout[k] + off;   // the fused stage writes q_{k+1} directly
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    sem_rk3 g = new (std::nothrow) sem_rk3_s();
    if (!g)
        return fail(SEM_ERR_NO_MEMORY, "graph allocation");
    g->fused = fused;
    PlanCore* c[3] = {nullptr, nullptr, nullptr};
    sem_status st = SEM_OK;
    for (int k = 0; k < 3 && st == SEM_OK; ++k) {
        const semk::RkStage rk{a[k], b[k], dt};
        st = build_plan(sb[k].data(), nblocks, dtype, phys, k == 0 ? flags : 0, s,
                        k == 0 ? nullptr : c[0], fused ? &rk : nullptr, fused ? xs.data() : nullptr,
                        &c[k]);
    }
    if (st != SEM_OK) {
        for (PlanCore* ck : c)
            if (ck) {
                free_core(ck);
                delete ck;
            }
        delete g;
        return st;
    }
    for (int k = 0; k < 3; ++k) {
        g->stage[k] = *c[k];
        delete c[k];
    }
    auto destroy_all = [&]() {
        for (PlanCore& ck : g->stage)
            free_core(&ck);
        if (g->exec)
            (void)hipGraphExecDestroy(g->exec);
        if (g->graph)
            (void)hipGraphDestroy(g->graph);
        delete g;
    };
    hipStream_t cs = nullptr;
    hipError_t err = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (err != hipSuccess) {
        destroy_all();
        return hip_fail(err, "capture stream");
    }
    err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    for (int k = 0; k < 3 && err == hipSuccess; ++k) {
        const PlanCore& ck = g->stage[k];
        err = launch(ck, ck.d_tiles, ck.ntiles, ck.lds_bytes, cs);
        if (err == hipSuccess && !fused) {
            if (dtype == SEM_F64)
                err = semh::launch_axpby<double>(n, a[k], static_cast<const double*>(q_n), b[k],
                                                 reinterpret_cast<const double*>(qin[k]), dt,
                                                 static_cast<const double*>(L),
                                                 reinterpret_cast<double*>(qout[k]), cs);
            else
                err = semh::launch_axpby<float>(n, a[k], static_cast<const float*>(q_n), b[k],
                                                reinterpret_cast<const float*>(qin[k]), dt,
                                                static_cast<const float*>(L),
                                                reinterpret_cast<float*>(qout[k]), cs);
        }
    }
    hipGraph_t graph = nullptr;
    hipError_t err_end = hipStreamEndCapture(cs, &graph);
    if (err == hipSuccess)
        err = err_end;
    g->graph = graph;
    if (err == hipSuccess)
        err = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (err != hipSuccess) {
        destroy_all();
        return hip_fail(err, "RK3 graph capture");
    }
    *out = g;
    return SEM_OK;
}

extern "C" sem_status sem_rk3_graph_launch(sem_rk3 step, void* stream)
{
    if (!step || !step->exec)
        return fail(SEM_ERR_INVALID_ARG, "step is NULL or destroyed");
    hipError_t err = hipGraphLaunch(step->exec, static_cast<hipStream_t>(stream));
    if (err != hipSuccess)
        return hip_fail(err, "hipGraphLaunch");
    return SEM_OK;
}

extern "C" sem_status sem_rk3_graph_describe(sem_rk3 step, char* buf, int32_t len)
{
    if (!step || !buf || len < 1)
        return fail(SEM_ERR_INVALID_ARG, "NULL step or buffer");
    std::string s = std::string("{\"fused_stages\": ") + (step->fused ? "true" : "false") +
                    ", \"stage_plan\": " + describe(step->stage[0]) + "}";
    snprintf(buf, (size_t)len, "%s", s.c_str());
    return SEM_OK;
}

extern "C" sem_status sem_rk3_graph_destroy(sem_rk3 step)
{
    if (!step)
        return fail(SEM_ERR_INVALID_ARG, "step is NULL");
    for (PlanCore& c : step->stage)
        free_core(&c);
    if (step->exec)
        (void)hipGraphExecDestroy(step->exec);
    if (step->graph)
        (void)hipGraphDestroy(step->graph);
    delete step;
    return SEM_OK;
}
