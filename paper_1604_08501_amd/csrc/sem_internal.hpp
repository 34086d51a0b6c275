// Internal host-side interface between the C-ABI layer (sem_api.cpp) and the
// kernel translation units.  Not installed; not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sem_device.hpp"

// Compiled tile shapes (Nq, elements per workgroup, layout).  The
// single-order kernels use ceil64(EPB * Nq^3) threads (one node per thread;
// 512 threads with two nodes each for aliased tiles of more than 512 nodes);
// the mixed-order batch kernel runs every shape with a fixed workgroup size.
// Layout 0 keeps all three directions' fluxes in LDS, layout 1 one direction
// at a time.
#define SEM_VARIANTS(X)                                                        \
    X(2, 8, 0) X(2, 16, 0) X(2, 32, 0) X(2, 64, 0) X(2, 128, 0)                \
    X(3, 4, 0) X(3, 8, 0) X(3, 16, 0) X(3, 32, 0)                              \
    X(4, 1, 0) X(4, 2, 0) X(4, 4, 0) X(4, 8, 0) X(4, 16, 0)                    \
    X(5, 1, 0) X(5, 2, 0) X(5, 4, 0) X(5, 8, 0)                                \
    X(6, 1, 0) X(6, 2, 0) X(6, 4, 0) X(6, 2, 1) X(6, 4, 1)                     \
    X(7, 1, 0) X(7, 2, 0) X(7, 1, 1) X(7, 2, 1)                                \
    X(8, 1, 0) X(8, 2, 0) X(8, 1, 1) X(8, 2, 1)                                \
    X(9, 1, 0) X(9, 1, 1)                                                      \
    X(10, 1, 0) X(10, 1, 1)

namespace semh {

// A dispatch's work-item count (workgroups x lanes) is a 32-bit field of the
// dispatch packet: launches beyond it fail with this error instead.
inline bool dispatch_fits(int64_t groups, int threads)
{
    return groups >= 1 && groups * (int64_t)threads <= (int64_t)UINT32_MAX;
}

struct VariantDef {
    int nq, epb, lay;
};
#define SEM_X_DEF(NQ_, EPB_, LAY_) VariantDef{NQ_, EPB_, LAY_},
inline constexpr VariantDef kVariants[] = {SEM_VARIANTS(SEM_X_DEF)};
#undef SEM_X_DEF
inline constexpr int kNumVariants = (int)(sizeof(kVariants) / sizeof(kVariants[0]));

constexpr int variant_index(int nq, int epb, int lay)
{
    for (int i = 0; i < kNumVariants; ++i)
        if (kVariants[i].nq == nq && kVariants[i].epb == epb && kVariants[i].lay == lay)
            return i;
    return -1;
}

constexpr int kMaxLdsBytes = 160 * 1024;   // LDS per CU on gfx950
constexpr int kBatchThreads[] = {256, 512, 1024};

// Single-order forward/adjoint launchers (defined per dtype in kernels_*.hip).
template <typename T>
hipError_t launch_volume(int nq, int epb, int lay, const semk::BlockPtrs<T>& B,
                         const semk::Phys& ph, int accumulate, hipStream_t s);
template <typename T>
hipError_t launch_adjoint(int nq, int epb, const semk::AdjPtrs<T>& B, const semk::Phys& ph,
                          int accumulate, hipStream_t s);
template <typename T>
hipError_t launch_axpby(int64_t n, double a, const T* x, double b, const T* y, double c,
                        const T* z, T* out, hipStream_t s);

// Extended volume term (defined per dtype in ext_*.hip): nf = 5 or 8 fields,
// dirs = 3 (r+s) or 7 (r+s+t), Nq in 2..10, 12, 16 where the LDS allows.
template <typename T>
bool ext_supported(int nq, int nf, int dirs);
template <typename T>
hipError_t launch_volume_ext(int nq, int nf, int dirs, const semk::BlockPtrs<T>& B,
                             const semk::Phys& ph, int accumulate, hipStream_t s);
// Volume term with per-element metric terms (affine elements; geo [Ne][10]),
// five fields, r+s+t, Nq in 2..10, 12, 16 where the LDS allows.
template <typename T>
bool affine_supported(int nq);
template <typename T>
hipError_t launch_volume_affine(int nq, const semk::BlockPtrs<T>& B, const semk::Phys& ph,
                                int accumulate, hipStream_t s);

// Surface term (surface_*.hip): Nq 2..10, 12, 16.
template <typename T>
bool surface_supported(int nq);
template <typename T>
hipError_t launch_surface(int nq, const semk::SurfPtrs<T>& B, const semk::Phys& ph, int accumulate,
                          hipStream_t s);

// Volume + surface term in one launch (rhs_*.hip): Nq 2..10.
template <typename T>
bool rhs_supported(int nq);
template <typename T>
hipError_t launch_volume_surface(int nq, const semk::BlockPtrs<T>& B, const int32_t* nbr,
                                 const semk::Phys& ph, int accumulate, hipStream_t s);

// Workgroup cap of the strided k-slice and t-column launches set by
// sem_set_max_workgroups (0 = none); one relaxed atomic load.
int64_t max_workgroups_cap();

// Optimisation ladder of the fused r+s, 8-field FP32 kernel (ladder.hip):
// levels 1..5, Nq 2..10, 12, 16.
bool ladder_supported(int nq);
hipError_t launch_ladder(int level, int nq, int64_t Ne, const float* D, const float* geo,
                         const float* q, float* rhs, const semk::Phys& ph, hipStream_t s);

// Mixed-order batch kernel (defined per dtype in batch_*.hip): one tile per
// workgroup.
struct Tile {
    int32_t block;
    int32_t variant;
    int32_t ne;
    int32_t pad;
    int64_t e0;
};
// rk: the shape must also run a fused Runge-Kutta stage (one node per thread
// for FULL, at most two for ALIAS)
template <typename T>
bool batch_variant_ok(int nt, int nq, int epb, int lay, bool rk);
template <typename T>
int batch_lds_bytes(int nt, int nq, int epb, int lay);
// rk = false: rhs = v(q); rk = true: every block runs the fused stage
// out = a x + b (q + dt v) with the coefficients of its descriptor.
template <typename T>
hipError_t launch_batch(int nt, const Tile* d_tiles, int ntiles,
                        const semk::BatchBlock<T>* d_blocks, bool rk, int lds_bytes,
                        hipStream_t s);
template <typename T>
hipError_t batch_blocks_per_cu(int nt, int lds_bytes, bool rk, int* out);

// Must run once per process before occupancy queries or launches (sets the
// dynamic-LDS limit of the batch kernels).
template <typename T>
hipError_t batch_prepare();

}  // namespace semh
