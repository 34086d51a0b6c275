// Host-side helpers shared by the C-ABI translation units (sem_api.cpp:
// single-order entry points; sem_plan.cpp: batch plans and the RK3 graph):
// status and error text, argument checks, built-in tile shapes.  Internal to
// libsem.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sem.h"
#include "sem_internal.hpp"

namespace semapi {

// Sets the thread's last-error text and returns st.
sem_status fail(sem_status st, const char* fmt, ...);
sem_status hip_fail(hipError_t err, const char* what);
const char* last_error();
// SEM_LOG=1 in the environment: autotuner decisions on stderr.
bool log_enabled();

size_t elem_size(sem_dtype dt);
semk::Phys to_phys(const sem_phys* p);

constexpr int kMinNq = 2, kMaxNq = 10;

// Historical small-order element counts (all fluxes resident).
int default_epb(int nq);

// Built-in single-order tile per (dtype, Nq): the fastest compiled shape
// measured on MI355X at about 1 GB per launch.
struct DefaultTile {
    int epb;
    int lay;
};
DefaultTile default_tile(sem_dtype dt, int nq);

// Built-in batch shape of order nq in a launch of nt threads (the shape a
// plan takes without autotuning); false if none fits.
bool batch_default_shape(sem_dtype dt, int nt, int nq, int* epb, int* lay);

sem_status check_dtype(sem_dtype dt);
sem_status check_order(int32_t Ne, int32_t Nq);
sem_status check_ptr(const void* p, size_t align, const char* name, bool required = true);
// A named device array and its extent in bytes (for overlap checks).
struct ByteRange {
    const char* name;
    const void* p;
    size_t bytes;
};
// True when the byte ranges [a, a + abytes) and [b, b + bbytes) intersect
// (NULL or empty ranges never do).
bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes);
// SEM_ERR_INVALID_ARG when the output range overlaps any input range.
sem_status check_output_overlap(const char* out_name, const void* out, size_t out_bytes,
                                const ByteRange* inputs, int n_inputs);

// Sizes of the arrays of a volume-term call: Ne elements of Nq^3 nodes, nf
// fields, geo_values_per_element metric values (10 Nq^3 per node, 10 for the
// per-element form).
struct VolumeExtent {
    int64_t Ne;
    int Nq;
    int nf;
    int64_t geo_values_per_element;
};
// Pointers, alignment, the reference pair, and rhs overlapping an input.
sem_status check_volume_ptrs(sem_dtype dt, const void* D, const void* geo, const void* q,
                             const void* rho_ref, const double* theta_ref, const sem_phys* phys,
                             const void* rhs, const VolumeExtent& x);
sem_status check_volume_args(int32_t Ne, int32_t Nq, sem_dtype dt, const void* D, const void* geo,
                             const void* q, const void* rho_ref, const double* theta_ref,
                             const sem_phys* phys, const void* rhs);

template <typename T>
semk::BlockPtrs<T> block_ptrs(int64_t Ne, const void* D, const void* geo, const void* q,
                              const void* rho_ref, const double* theta_ref, void* rhs)
{
    return semk::BlockPtrs<T>{static_cast<const T*>(D),   static_cast<const T*>(geo),
                              static_cast<const T*>(q),   static_cast<const T*>(rho_ref),
                              theta_ref,                  static_cast<T*>(rhs),
                              Ne,                         nullptr};
}

}  // namespace semapi

#define SEM_TRY(expr)                 \
    do {                              \
        sem_status _st = (expr);      \
        if (_st != SEM_OK)            \
            return _st;               \
    } while (0)
