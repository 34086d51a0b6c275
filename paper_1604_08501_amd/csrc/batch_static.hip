// Mixed-order batch evaluated without any device allocation, for callers
// that cannot allocate (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  The tile and block tables that a plan
// keeps in memory it allocates live here in one file-scope device array,
// `scratch`, which every call on a GPU shares; a small fill kernel, whose
// arguments carry the block descriptors, writes them before the batch kernel
// of sem_batch_execute runs on them.
//
// The host code never passes `scratch` itself to a kernel or a copy: in host
// code that name is a stand-in, not a device address.  The device address of
// each GPU's copy is taken once per device with hipGetSymbolAddress and kept
// in g_scratch_ptr.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>

#include "sem.h"
#include "sem_host.hpp"
#include "sem_internal.hpp"

namespace {

constexpr int kMaxBlocks = SEM_STATIC_MAX_BLOCKS;
constexpr int kMaxTiles = SEM_STATIC_MAX_TILES;
// block table first (the larger of the two dtypes' descriptors), then tiles
constexpr size_t kBlockBytes = std::max(sizeof(semk::BatchBlock<double>),
                                        sizeof(semk::BatchBlock<float>));
constexpr size_t kTileOffset = ((kMaxBlocks * kBlockBytes + 255) / 256) * 256;
constexpr size_t kScratchBytes = kTileOffset + (size_t)kMaxTiles * sizeof(semh::Tile);

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Descriptors of one call, by value: blocks in tile order (decreasing cost
// per tile), the first tile of each block and its tile shape.
template <typename T>
struct FillArgs {
    semk::BatchBlock<T> blocks[kMaxBlocks];
    int64_t first_tile[kMaxBlocks + 1];
    int32_t variant[kMaxBlocks];
    int32_t epb[kMaxBlocks];
    int32_t nblocks;
};

template <typename T>
__global__ __launch_bounds__(256) void fill_tables(FillArgs<T> a, unsigned char* base)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    auto* blocks = reinterpret_cast<semk::BatchBlock<T>*>(base);
    auto* tiles = reinterpret_cast<semh::Tile*>(base + kTileOffset);
    if (t < a.nblocks)
        blocks[t] = a.blocks[t];
    if (t >= a.first_tile[a.nblocks])
        return;
    int b = 0;
    while (t >= a.first_tile[b + 1])
        ++b;
    const int64_t e0 = (t - a.first_tile[b]) * a.epb[b];
    const int64_t left = a.blocks[b].b.Ne - e0;
    tiles[t] = semh::Tile{b, a.variant[b], (int32_t)std::min<int64_t>(a.epb[b], left), 0, e0};
}

// Per-device address of `scratch`, taken once per device with that device
// current; the dynamic-LDS limit of the batch kernels is raised at the same
// time.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

sem_status device_scratch(void** out)
{
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess)
        return semapi::hip_fail(err, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return semapi::fail(SEM_ERR_UNSUPPORTED, "device %d beyond the %d this library tracks", dev,
                            kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (err != hipSuccess)
            return semapi::hip_fail(err, "hipGetSymbolAddress(scratch)");
        err = semh::batch_prepare<double>();
        if (err == hipSuccess)
            err = semh::batch_prepare<float>();
        if (err != hipSuccess)
            return semapi::hip_fail(err, "batch kernel setup");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SEM_OK;
}

template <typename T>
sem_status run(const sem_block* blocks, int32_t nblocks, const sem_phys* phys, hipStream_t s)
{
    using semapi::fail;
    const sem_dtype dt = sizeof(T) == 8 ? SEM_F64 : SEM_F32;
    // built-in shapes: the smallest workgroup size for which every order has one
    int nt = 0;
    int epb[kMaxBlocks], lay[kMaxBlocks];
    for (int cand : semh::kBatchThreads) {
        bool all = true;
        for (int i = 0; i < nblocks && all; ++i)
            all = semapi::batch_default_shape(dt, cand, blocks[i].Nq, &epb[i], &lay[i]);
        if (all) {
            nt = cand;
            break;
        }
    }
    if (!nt)
        return fail(SEM_ERR_UNSUPPORTED, "no built-in batch shape covers every order of the call");
    // tile order: blocks by decreasing cost per tile (nodes per tile), ties in
    // call order, as the tile table of a plan without autotuning
    int order[kMaxBlocks];
    for (int i = 0; i < nblocks; ++i)
        order[i] = i;
    auto cost = [&](int i) { return (double)blocks[i].Nq * blocks[i].Nq * blocks[i].Nq * epb[i]; };
    std::stable_sort(order, order + nblocks, [&](int x, int y) { return cost(x) > cost(y); });
    FillArgs<T> a{};
    a.nblocks = nblocks;
    a.first_tile[0] = 0;
    const semk::Phys ph = semapi::to_phys(phys);
    int lds = 0;
    for (int k = 0; k < nblocks; ++k) {
        const sem_block& b = blocks[order[k]];
        a.blocks[k] = semk::BatchBlock<T>{
            semapi::block_ptrs<T>(b.Ne, b.D, b.geo, b.q, b.rho_ref, b.theta_ref, b.rhs), ph,
            semk::RkStage{0.0, 0.0, 0.0}};
        a.variant[k] = semh::variant_index(b.Nq, epb[order[k]], lay[order[k]]);
        a.epb[k] = epb[order[k]];
        a.first_tile[k + 1] = a.first_tile[k] + (b.Ne + epb[order[k]] - 1) / epb[order[k]];
        lds = std::max(lds, semh::batch_lds_bytes<T>(nt, b.Nq, epb[order[k]], lay[order[k]]));
    }
    const int64_t ntiles = a.first_tile[nblocks];
    if (ntiles > kMaxTiles)
        return fail(SEM_ERR_INVALID_ARG,
                    "%lld tiles exceed the static tile table (%d tiles); use sem_batch_plan",
                    (long long)ntiles, kMaxTiles);
    void* ptr = nullptr;
    SEM_TRY(device_scratch(&ptr));
    int per_cu = 0;
    hipError_t err = semh::batch_blocks_per_cu<T>(nt, lds, false, &per_cu);
    if (err != hipSuccess)
        return semapi::hip_fail(err, "occupancy query");
    if (per_cu < 1)
        return fail(SEM_ERR_UNSUPPORTED, "batch kernel cannot be resident with %d B of LDS", lds);
    auto* base = static_cast<unsigned char*>(ptr);
    const unsigned fill_grid = (unsigned)((ntiles + 255) / 256);
    hipLaunchKernelGGL(fill_tables<T>, dim3(fill_grid), dim3(256), 0, s, a, base);
    err = hipGetLastError();
    if (err != hipSuccess)
        return semapi::hip_fail(err, "tile table fill launch");
    err = semh::launch_batch<T>(nt, reinterpret_cast<const semh::Tile*>(base + kTileOffset),
                                (int)ntiles,
                                reinterpret_cast<const semk::BatchBlock<T>*>(base), false, lds, s);
    if (err != hipSuccess)
        return semapi::hip_fail(err, "batch kernel launch");
    return SEM_OK;
}

}  // namespace

extern "C" sem_status sem_batch_rhs_static(const sem_block* blocks, int32_t nblocks,
                                           sem_dtype dtype, const sem_phys* phys, void* stream)
{
    using semapi::fail;
    SEM_TRY(semapi::check_dtype(dtype));
    if (!blocks || nblocks < 1)
        return fail(SEM_ERR_INVALID_ARG, "need at least one block (nblocks = %d)", nblocks);
    if (nblocks > kMaxBlocks)
        return fail(SEM_ERR_INVALID_ARG, "%d blocks exceed the static block table (%d blocks)",
                    nblocks, kMaxBlocks);
    if (!phys)
        return fail(SEM_ERR_INVALID_ARG, "phys is NULL");
    for (int i = 0; i < nblocks; ++i) {
        const sem_block& b = blocks[i];
        sem_status st = semapi::check_volume_args(b.Ne, b.Nq, dtype, b.D, b.geo, b.q, b.rho_ref,
                                                  b.theta_ref, phys, b.rhs);
        if (st != SEM_OK) {
            char msg[256];
            snprintf(msg, sizeof msg, "%s", semapi::last_error());
            return fail(st, "block %d: %s", i, msg);
        }
    }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    return dtype == SEM_F64 ? run<double>(blocks, nblocks, phys, s)
                            : run<float>(blocks, nblocks, phys, s);
}
