// C-ABI of libsem.so, single-order entry points: argument validation, status
// codes, tile selection and the launches of the volume, extended, affine,
// ladder, adjoint and axpby kernels.  Batch plans and the RK3 graph are in
// sem_plan.cpp.  The operations themselves are documented in include/sem.h.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "sem.h"
#include "sem_host.hpp"
#include "sem_internal.hpp"

namespace semapi {

namespace {
thread_local std::string g_last_error;
}  // namespace

const char* last_error() { return g_last_error.c_str(); }

sem_status fail(sem_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

sem_status hip_fail(hipError_t err, const char* what)
{
    return fail(SEM_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(err), (int)err);
}

bool log_enabled()
{
    static int on = -1;
    if (on < 0) {
        const char* v = getenv("SEM_LOG");
        on = (v && *v && strcmp(v, "0") != 0) ? 1 : 0;
    }
    return on == 1;
}

size_t elem_size(sem_dtype dt) { return dt == SEM_F64 ? 8 : 4; }

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

semk::Phys to_phys(const sem_phys* p)
{
    return semk::Phys{p->p0, p->gamma, p->R, p->grav, p->R / p->p0};
}

// Element counts of the small-order shapes with all fluxes resident: the
// batch's fallback when a default tile does not fit its launch, and the
// adjoint's tile.
int default_epb(int nq)
{
    switch (nq) {
    case 2: return 32;
    case 3: return 8;
    case 4: return 4;
    case 5: return 2;
    default: return 1;
    }
}

// public layout code (sem_tile.layout) -> internal layout, -1 if unknown
// Every shape moves the same bytes; they differ in occupancy and barrier
// count.
DefaultTile default_tile(sem_dtype dt, int nq)
{
    const bool f64 = dt == SEM_F64;
    switch (nq) {
    case 2: return {f64 ? 64 : 128, semk::FULL};
    case 3: return {f64 ? 8 : 16, semk::FULL};
    case 4: return {f64 ? 8 : 2, semk::FULL};
    case 5: return {2, semk::FULL};
    case 6: return {4, semk::ALIAS};
    case 7: return {f64 ? 2 : 1, semk::ALIAS};
    case 8: return {f64 ? 2 : 1, semk::ALIAS};
    default: return {1, semk::ALIAS};   // 9, 10
    }
}

// The compiled shape with the smallest element count for (nq, lay), or -1.
int smallest_epb(int nq, int lay)
{
    int best = -1;
    for (int i = 0; i < semh::kNumVariants; ++i) {
        const semh::VariantDef v = semh::kVariants[i];
        if (v.nq == nq && v.lay == lay && (best < 0 || v.epb < best))
            best = v.epb;
    }
    return best;
}

int internal_layout(int32_t code)
{
    switch (code) {
    case SEM_LAYOUT_DEFAULT:
    case SEM_LAYOUT_FULL: return semk::FULL;
    case SEM_LAYOUT_ALIAS: return semk::ALIAS;
    default: return -1;
    }
}

int32_t public_layout(int lay) { return lay == semk::ALIAS ? SEM_LAYOUT_ALIAS : SEM_LAYOUT_FULL; }

sem_status check_dtype(sem_dtype dt)
{
    if (dt != SEM_F64 && dt != SEM_F32)
        return fail(SEM_ERR_INVALID_ARG, "unknown dtype %d", (int)dt);
    return SEM_OK;
}

sem_status check_order(int32_t Ne, int32_t Nq)
{
    if (Ne < 1)
        return fail(SEM_ERR_INVALID_ARG, "Ne = %d: at least one element is required", Ne);
    if (Nq < kMinNq || Nq > kMaxNq)
        return fail(SEM_ERR_UNSUPPORTED, "Nq = %d is not compiled (supported %d..%d)", Nq, kMinNq,
                    kMaxNq);
    return SEM_OK;
}

sem_status check_ptr(const void* p, size_t align, const char* name, bool required)
{
    if (!p)
        return required ? fail(SEM_ERR_INVALID_ARG, "%s is NULL", name) : SEM_OK;
    if (!aligned(p, align))
        return fail(SEM_ERR_INVALID_ARG, "%s = %p is not %zu-byte aligned", name, p, align);
    return SEM_OK;
}

bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes)
{
    if (!a || !b || abytes == 0 || bbytes == 0)
        return false;
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

sem_status check_output_overlap(const char* out_name, const void* out, size_t out_bytes,
                                const ByteRange* inputs, int n_inputs)
{
    for (int i = 0; i < n_inputs; ++i)
        if (ranges_overlap(out, out_bytes, inputs[i].p, inputs[i].bytes))
            return fail(SEM_ERR_INVALID_ARG, "%s [%p, +%zu B) overlaps %s [%p, +%zu B)", out_name,
                        out, out_bytes, inputs[i].name, inputs[i].p, inputs[i].bytes);
    return SEM_OK;
}

sem_status check_volume_ptrs(sem_dtype dt, const void* D, const void* geo, const void* q,
                             const void* rho_ref, const double* theta_ref, const sem_phys* phys,
                             const void* rhs, const VolumeExtent& x)
{
    if (!phys)
        return fail(SEM_ERR_INVALID_ARG, "phys is NULL");
    const size_t es = elem_size(dt);
    SEM_TRY(check_ptr(D, es, "D"));
    SEM_TRY(check_ptr(geo, es, "geo"));
    SEM_TRY(check_ptr(q, es, "q"));
    SEM_TRY(check_ptr(rhs, es, "rhs"));
    if ((rho_ref == nullptr) != (theta_ref == nullptr))
        return fail(SEM_ERR_INVALID_ARG, "rho_ref and theta_ref must both be NULL or both be given");
    SEM_TRY(check_ptr(rho_ref, es, "rho_ref", false));
    SEM_TRY(check_ptr(theta_ref, 8, "theta_ref", false));
    // rhs is written while every input is read: no byte of it may lie in an input
    const size_t M = (size_t)x.Nq * x.Nq * x.Nq;
    const size_t Ne = (size_t)x.Ne;
    const ByteRange in[] = {
        {"D", D, (size_t)x.Nq * x.Nq * es},
        {"geo", geo, Ne * (size_t)x.geo_values_per_element * es},
        {"q", q, Ne * (size_t)x.nf * M * es},
        {"rho_ref", rho_ref, Ne * M * es},
        {"theta_ref", theta_ref, Ne * M * 8},
    };
    return check_output_overlap("rhs", rhs, Ne * (size_t)x.nf * M * es, in, 5);
}

sem_status check_volume_args(int32_t Ne, int32_t Nq, sem_dtype dt, const void* D, const void* geo,
                             const void* q, const void* rho_ref, const double* theta_ref,
                             const sem_phys* phys, const void* rhs)
{
    SEM_TRY(check_dtype(dt));
    SEM_TRY(check_order(Ne, Nq));
    return check_volume_ptrs(dt, D, geo, q, rho_ref, theta_ref, phys, rhs,
                             VolumeExtent{Ne, Nq, 5, 10 * (int64_t)Nq * Nq * Nq});
}

}  // namespace semapi

using namespace semapi;

namespace {

int tile_options(int nq, sem_tile* out, int cap)
{
    int n = 0;
    for (int i = 0; i < semh::kNumVariants; ++i)
        if (semh::kVariants[i].nq == nq) {
            if (n < cap && out)
                out[n] = sem_tile{semh::kVariants[i].epb, public_layout(semh::kVariants[i].lay)};
            ++n;
        }
    return n;
}

}  // namespace

// ===========================================================================
// Single-order entry points
// ===========================================================================
extern "C" const char* sem_last_error(void) { return last_error(); }

extern "C" const char* sem_version(void) { return "semvol 0.2.0 (gfx950)"; }

namespace {
std::atomic<int64_t> g_max_workgroups{0};
}  // namespace

int64_t semh::max_workgroups_cap() { return g_max_workgroups.load(std::memory_order_relaxed); }

extern "C" sem_status sem_set_max_workgroups(int64_t cap)
{
    if (cap < 0)
        return fail(SEM_ERR_INVALID_ARG, "cap = %lld < 0", (long long)cap);
    g_max_workgroups.store(cap, std::memory_order_relaxed);
    return SEM_OK;
}

extern "C" int32_t sem_tile_options(sem_dtype dtype, int32_t Nq, sem_tile* out, int32_t cap)
{
    if (dtype != SEM_F64 && dtype != SEM_F32)
        return 0;   // every compiled shape exists for both dtypes
    return tile_options(Nq, out, cap);
}

extern "C" sem_status sem_volume_rhs_tiled(int32_t Ne, int32_t Nq, sem_dtype dtype, const void* D,
                                           const void* geo, const void* q, const void* rho_ref,
                                           const double* theta_ref, const sem_phys* phys, void* rhs,
                                           int32_t accumulate, const sem_tile* tile, void* stream)
{
    SEM_TRY(check_volume_args(Ne, Nq, dtype, D, geo, q, rho_ref, theta_ref, phys, rhs));
    const int32_t code = tile ? tile->layout : SEM_LAYOUT_DEFAULT;
    if (internal_layout(code) < 0)
        return fail(SEM_ERR_INVALID_ARG, "unknown tile layout %d", code);
    const DefaultTile dft = default_tile(dtype, Nq);
    int epb = tile && tile->elems_per_block > 0 ? tile->elems_per_block : 0;
    int lay = code == SEM_LAYOUT_DEFAULT ? -1 : internal_layout(code);
    if (epb == 0 && lay < 0) {
        epb = dft.epb;
        lay = dft.lay;
    } else if (epb == 0) {
        epb = semh::variant_index(Nq, dft.epb, lay) >= 0 ? dft.epb : smallest_epb(Nq, lay);
    } else if (lay < 0) {
        lay = semh::variant_index(Nq, epb, semk::FULL) >= 0 ? semk::FULL : semk::ALIAS;
    }
    if (semh::variant_index(Nq, epb, lay) < 0)
        return fail(SEM_ERR_UNSUPPORTED,
                    "tile (elems_per_block = %d, layout = %d) is not compiled for Nq = %d", epb,
                    (int)public_layout(lay), Nq);
    const semk::Phys ph = to_phys(phys);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t err;
    if (dtype == SEM_F64)
        err = semh::launch_volume<double>(
            Nq, epb, lay, block_ptrs<double>(Ne, D, geo, q, rho_ref, theta_ref, rhs), ph, accumulate,
            s);
    else
        err = semh::launch_volume<float>(
            Nq, epb, lay, block_ptrs<float>(Ne, D, geo, q, rho_ref, theta_ref, rhs), ph, accumulate,
            s);
    if (err != hipSuccess)
        return hip_fail(err, "volume kernel launch");
    return SEM_OK;
}

extern "C" sem_status sem_volume_rhs(int32_t Ne, int32_t Nq, sem_dtype dtype, const void* D,
                                     const void* geo, const void* q, const void* rho_ref,
                                     const double* theta_ref, const sem_phys* phys, void* rhs,
                                     int32_t accumulate, void* stream)
{
    return sem_volume_rhs_tiled(Ne, Nq, dtype, D, geo, q, rho_ref, theta_ref, phys, rhs, accumulate,
                                nullptr, stream);
}

extern "C" sem_status sem_volume_rhs_ext(int32_t Ne, int32_t Nq, sem_dtype dtype, int32_t nfields,
                                         uint32_t dirs, const void* D, const void* geo,
                                         const void* q, const void* rho_ref,
                                         const double* theta_ref, const sem_phys* phys, void* rhs,
                                         int32_t accumulate, void* stream)
{
    SEM_TRY(check_dtype(dtype));
    if (Ne < 1)
        return fail(SEM_ERR_INVALID_ARG, "Ne = %d: at least one element is required", Ne);
    if (nfields != 5 && nfields != 8)
        return fail(SEM_ERR_UNSUPPORTED, "nfields = %d (5, or 8 with the passive tracers)", nfields);
    if (dirs != (SEM_DIR_R | SEM_DIR_S) && dirs != (SEM_DIR_R | SEM_DIR_S | SEM_DIR_T))
        return fail(SEM_ERR_UNSUPPORTED, "dirs = %u (r+s = 3 or r+s+t = 7)", dirs);
    const bool ok = dtype == SEM_F64 ? semh::ext_supported<double>(Nq, nfields, (int)dirs)
                                     : semh::ext_supported<float>(Nq, nfields, (int)dirs);
    if (!ok)
        return fail(SEM_ERR_UNSUPPORTED,
                    "Nq = %d with %d fields and dirs = %u is not compiled for this dtype "
                    "(Nq 2..10, 12, 16)", Nq, nfields, dirs);
    SEM_TRY(check_volume_ptrs(dtype, D, geo, q, rho_ref, theta_ref, phys, rhs,
                              VolumeExtent{Ne, Nq, nfields, 10 * (int64_t)Nq * Nq * Nq}));
    if (nfields == 5 && dirs == 7 && Nq <= kMaxNq)
        return sem_volume_rhs(Ne, Nq, dtype, D, geo, q, rho_ref, theta_ref, phys, rhs, accumulate,
                              stream);
    const semk::Phys ph = to_phys(phys);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t err;
    if (dtype == SEM_F64)
        err = semh::launch_volume_ext<double>(
            Nq, nfields, (int)dirs, block_ptrs<double>(Ne, D, geo, q, rho_ref, theta_ref, rhs), ph,
            accumulate, s);
    else
        err = semh::launch_volume_ext<float>(
            Nq, nfields, (int)dirs, block_ptrs<float>(Ne, D, geo, q, rho_ref, theta_ref, rhs), ph,
            accumulate, s);
    if (err != hipSuccess)
        return hip_fail(err, "extended volume kernel launch");
    return SEM_OK;
}

extern "C" sem_status sem_volume_rhs_ladder(int32_t level, int32_t Ne, int32_t Nq, const void* D,
                                            const void* geo, const void* q, const sem_phys* phys,
                                            void* rhs, void* stream)
{
    if (level < 1 || level > SEM_LADDER_LEVELS)
        return fail(SEM_ERR_INVALID_ARG, "level = %d (1..%d)", level, SEM_LADDER_LEVELS);
    if (Ne < 1)
        return fail(SEM_ERR_INVALID_ARG, "Ne = %d: at least one element is required", Ne);
    if (!semh::ladder_supported(Nq) || !semh::ext_supported<float>(Nq, 8, 3))
        return fail(SEM_ERR_UNSUPPORTED, "Nq = %d is not compiled (Nq 2..10, 12, 16)", Nq);
    SEM_TRY(check_volume_ptrs(SEM_F32, D, geo, q, nullptr, nullptr, phys, rhs,
                              VolumeExtent{Ne, Nq, 8, 10 * (int64_t)Nq * Nq * Nq}));
    if (phys->grav != 0.0)
        return fail(SEM_ERR_UNSUPPORTED,
                    "grav = %g: the benchmark kernel has no source term (grav must be 0)", phys->grav);
    if (level == SEM_LADDER_LEVELS)
        return sem_volume_rhs_ext(Ne, Nq, SEM_F32, 8, SEM_DIR_R | SEM_DIR_S, D, geo, q, nullptr,
                                  nullptr, phys, rhs, 1, stream);
    const hipError_t err = semh::launch_ladder(
        level, Nq, Ne, static_cast<const float*>(D), static_cast<const float*>(geo),
        static_cast<const float*>(q), static_cast<float*>(rhs), to_phys(phys),
        static_cast<hipStream_t>(stream));
    if (err != hipSuccess)
        return hip_fail(err, "ladder kernel launch");
    return SEM_OK;
}

extern "C" sem_status sem_volume_rhs_affine(int32_t Ne, int32_t Nq, sem_dtype dtype, const void* D,
                                            const void* geo_elem, const void* q,
                                            const void* rho_ref, const double* theta_ref,
                                            const sem_phys* phys, void* rhs, int32_t accumulate,
                                            void* stream)
{
    SEM_TRY(check_dtype(dtype));
    if (Ne < 1)
        return fail(SEM_ERR_INVALID_ARG, "Ne = %d: at least one element is required", Ne);
    const bool ok = dtype == SEM_F64 ? semh::affine_supported<double>(Nq)
                                     : semh::affine_supported<float>(Nq);
    if (!ok)
        return fail(SEM_ERR_UNSUPPORTED, "Nq = %d is not compiled for per-element metric terms "
                                         "in this dtype (Nq 2..10, 12, 16)",
                    Nq);
    SEM_TRY(check_volume_ptrs(dtype, D, geo_elem, q, rho_ref, theta_ref, phys, rhs,
                              VolumeExtent{Ne, Nq, 5, 10}));
    const semk::Phys ph = to_phys(phys);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t err;
    if (dtype == SEM_F64)
        err = semh::launch_volume_affine<double>(
            Nq, block_ptrs<double>(Ne, D, geo_elem, q, rho_ref, theta_ref, rhs), ph, accumulate, s);
    else
        err = semh::launch_volume_affine<float>(
            Nq, block_ptrs<float>(Ne, D, geo_elem, q, rho_ref, theta_ref, rhs), ph, accumulate, s);
    if (err != hipSuccess)
        return hip_fail(err, "affine volume kernel launch");
    return SEM_OK;
}

extern "C" sem_status sem_volume_rhs_adjoint(int32_t Ne, int32_t Nq, sem_dtype dtype, const void* D,
                                             const void* geo, const void* q, const sem_phys* phys,
                                             const void* lambda, void* mu, int32_t accumulate,
                                             void* stream)
{
    SEM_TRY(check_dtype(dtype));
    SEM_TRY(check_order(Ne, Nq));
    if (!phys)
        return fail(SEM_ERR_INVALID_ARG, "phys is NULL");
    const size_t es = elem_size(dtype);
    SEM_TRY(check_ptr(D, es, "D"));
    SEM_TRY(check_ptr(geo, es, "geo"));
    SEM_TRY(check_ptr(q, es, "q"));
    SEM_TRY(check_ptr(lambda, es, "lambda"));
    SEM_TRY(check_ptr(mu, es, "mu"));
    {
        const size_t M = (size_t)Nq * Nq * Nq;
        const ByteRange in[] = {
            {"D", D, (size_t)Nq * Nq * es},
            {"geo", geo, (size_t)Ne * 10 * M * es},
            {"q", q, (size_t)Ne * 5 * M * es},
            {"lambda", lambda, (size_t)Ne * 5 * M * es},
        };
        SEM_TRY(check_output_overlap("mu", mu, (size_t)Ne * 5 * M * es, in, 4));
    }
    const int epb = default_epb(Nq);
    const semk::Phys ph = to_phys(phys);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t err;
    if (dtype == SEM_F64)
        err = semh::launch_adjoint<double>(
            Nq, epb,
            semk::AdjPtrs<double>{static_cast<const double*>(D), static_cast<const double*>(geo),
                                  static_cast<const double*>(q), static_cast<const double*>(lambda),
                                  static_cast<double*>(mu), Ne},
            ph, accumulate, s);
    else
        err = semh::launch_adjoint<float>(
            Nq, epb,
            semk::AdjPtrs<float>{static_cast<const float*>(D), static_cast<const float*>(geo),
                                 static_cast<const float*>(q), static_cast<const float*>(lambda),
                                 static_cast<float*>(mu), Ne},
            ph, accumulate, s);
    if (err != hipSuccess)
        return hip_fail(err, "adjoint kernel launch");
    return SEM_OK;
}

extern "C" sem_status sem_surface_rhs(int32_t Ne, int32_t Nq, sem_dtype dtype, const int32_t* nbr,
                                      const void* geo, const void* q, const double* theta_ref,
                                      const sem_phys* phys, void* rhs, int32_t accumulate,
                                      void* stream)
{
    SEM_TRY(check_dtype(dtype));
    if (Ne < 1)
        return fail(SEM_ERR_INVALID_ARG, "Ne = %d: at least one element is required", Ne);
    const bool ok = dtype == SEM_F64 ? semh::surface_supported<double>(Nq)
                                     : semh::surface_supported<float>(Nq);
    if (!ok)
        return fail(SEM_ERR_UNSUPPORTED, "Nq = %d is not compiled for the surface term "
                                         "(Nq 2..10, 12, 16)", Nq);
    if (!phys)
        return fail(SEM_ERR_INVALID_ARG, "phys is NULL");
    const size_t es = elem_size(dtype);
    SEM_TRY(check_ptr(nbr, 4, "nbr"));
    SEM_TRY(check_ptr(geo, es, "geo"));
    SEM_TRY(check_ptr(q, es, "q"));
    SEM_TRY(check_ptr(theta_ref, 8, "theta_ref", false));
    SEM_TRY(check_ptr(rhs, es, "rhs"));
    {
        const size_t M = (size_t)Nq * Nq * Nq;
        const ByteRange in[] = {
            {"nbr", nbr, (size_t)Ne * 6 * 4},
            {"geo", geo, (size_t)Ne * 10 * M * es},
            {"q", q, (size_t)Ne * 5 * M * es},
            {"theta_ref", theta_ref, (size_t)Ne * M * 8},
        };
        SEM_TRY(check_output_overlap("rhs", rhs, (size_t)Ne * 5 * M * es, in, 4));
    }
    const semk::Phys ph = to_phys(phys);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t err;
    if (dtype == SEM_F64)
        err = semh::launch_surface<double>(
            Nq, semk::SurfPtrs<double>{nbr, static_cast<const double*>(geo),
                                       static_cast<const double*>(q), theta_ref,
                                       static_cast<double*>(rhs), Ne},
            ph, accumulate, s);
    else
        err = semh::launch_surface<float>(
            Nq, semk::SurfPtrs<float>{nbr, static_cast<const float*>(geo),
                                      static_cast<const float*>(q), theta_ref,
                                      static_cast<float*>(rhs), Ne},
            ph, accumulate, s);
    if (err != hipSuccess)
        return hip_fail(err, "surface kernel launch");
    return SEM_OK;
}

extern "C" sem_status sem_axpby(int64_t n, sem_dtype dtype, double a, const void* x, double b,
                                const void* y, double c, const void* z, void* out, void* stream)
{
    SEM_TRY(check_dtype(dtype));
    if (n < 0)
        return fail(SEM_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
    const size_t es = elem_size(dtype);
    SEM_TRY(check_ptr(x, es, "x", a != 0.0));
    SEM_TRY(check_ptr(y, es, "y"));
    SEM_TRY(check_ptr(z, es, "z"));
    SEM_TRY(check_ptr(out, es, "out"));
    // each value is read and written by one thread, so out may coincide with
    // an input; a shifted overlap would race
    {
        const size_t bytes = (size_t)n * es;
        const ByteRange in[] = {{"x", a != 0.0 ? x : nullptr, bytes}, {"y", y, bytes}, {"z", z, bytes}};
        for (const ByteRange& r : in)
            if (r.p != out)
                SEM_TRY(check_output_overlap("out", out, bytes, &r, 1));
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t err;
    if (dtype == SEM_F64)
        err = semh::launch_axpby<double>(n, a, static_cast<const double*>(x), b,
                                         static_cast<const double*>(y), c,
                                         static_cast<const double*>(z), static_cast<double*>(out), s);
    else
        err = semh::launch_axpby<float>(n, a, static_cast<const float*>(x), b,
                                        static_cast<const float*>(y), c,
                                        static_cast<const float*>(z), static_cast<float*>(out), s);
    if (err != hipSuccess)
        return hip_fail(err, "axpby kernel launch");
    return SEM_OK;
}

// ===========================================================================
// Batch plans
// ===========================================================================

extern "C" sem_status sem_rhs(int32_t Ne, int32_t Nq, sem_dtype dtype, const void* D,
                              const void* geo, const void* q, const void* rho_ref,
                              const double* theta_ref, const int32_t* nbr, const sem_phys* phys,
                              void* rhs, int32_t accumulate, void* stream)
{
    SEM_TRY(check_volume_args(Ne, Nq, dtype, D, geo, q, rho_ref, theta_ref, phys, rhs));
    const bool ok = dtype == SEM_F64 ? semh::rhs_supported<double>(Nq)
                                     : semh::rhs_supported<float>(Nq);
    if (!ok)
        return fail(SEM_ERR_UNSUPPORTED, "Nq = %d is not compiled for the whole rate (Nq 2..10)",
                    Nq);
    SEM_TRY(check_ptr(nbr, 4, "nbr"));
    {
        const ByteRange in[] = {{"nbr", nbr, (size_t)Ne * 6 * 4}};
        SEM_TRY(check_output_overlap("rhs", rhs, (size_t)Ne * 5 * Nq * Nq * Nq * elem_size(dtype),
                                     in, 1));
    }
    const semk::Phys ph = to_phys(phys);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t err =
        dtype == SEM_F64
            ? semh::launch_volume_surface<double>(
                  Nq, block_ptrs<double>(Ne, D, geo, q, rho_ref, theta_ref, rhs), nbr, ph,
                  accumulate, s)
            : semh::launch_volume_surface<float>(
                  Nq, block_ptrs<float>(Ne, D, geo, q, rho_ref, theta_ref, rhs), nbr, ph,
                  accumulate, s);
    if (err != hipSuccess)
        return hip_fail(err, "volume + surface kernel launch");
    return SEM_OK;
}
