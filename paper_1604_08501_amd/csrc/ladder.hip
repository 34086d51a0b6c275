// Optimisation ladder of the paper's benchmark kernel on gfx950 (the
// analogue of Sec. 4, Table 1): the fused r+s volume term with 8 fields in
// FP32, rhs accumulated (rhs += v), written at successive levels of
// optimisation so that each step's effect can be measured on its own.
//
// Levels 1-5 share the paper's work mapping: one workgroup per element, one
// lane per (i, j) node of a k-slice, k walked sequentially.
//   1  naive: for every output node, direction and n, the state and metric
//      terms at the line node are read from global memory, the pressure and
//      the flux are evaluated there, D is read from global memory, and rhs is
//      read, updated and written back in global memory (the listed kernels'
//      semantics: 2 Nq updates of every output);
//   2  D staged in LDS once per workgroup;
//   3  flux precompute: every node's two contravariant fluxes are evaluated
//      once per k-slice into LDS (the state is read once);
//   4  rhs accumulated in registers and updated in global memory once;
//   5  1/J applied once per output (distributive law).
// Level 6 is the production kernel of the extended volume term (node per
// thread over whole elements, shapes chosen at compile time).
//
// Levels 1-3 update rhs through volatile accesses, so that the compiler
// performs every memory update the level stands for instead of promoting rhs
// to a register.
#include "sem_internal.hpp"

#define SEM_LADDER_NQ(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(12) X(16)

namespace semk {

constexpr int kLadderFields = 8;

template <int NQ>
constexpr int ladder_threads()
{
    return ((NQ * NQ + 63) / 64) * 64;
}

// Contravariant flux of direction d (0 = r, 1 = s) at node m of one element,
// all eight fields, from the element's state qe and metric terms ge.
template <int M>
__device__ __forceinline__ void ladder_flux(const float* qe, const float* ge, int m, int d,
                                            const Phys& ph, float (&F)[kLadderFields])
{
    const float rho = qe[m], U1 = qe[M + m], U2 = qe[2 * M + m], U3 = qe[3 * M + m];
    const float Th = qe[4 * M + m];
    const float g1 = ge[(3 * d) * M + m], g2 = ge[(3 * d + 1) * M + m], g3 = ge[(3 * d + 2) * M + m];
    const float p = Pressure<float>::eval(Th, false, 0.0, ph);
    const float Ud = g1 * U1 + g2 * U2 + g3 * U3;
    const float vd = Ud / rho;
    F[0] = Ud;
    F[1] = U1 * vd + g1 * p;
    F[2] = U2 * vd + g2 * p;
    F[3] = U3 * vd + g3 * p;
    F[4] = Th * vd;
#pragma unroll
    for (int b = 5; b < kLadderFields; ++b)
        F[b] = qe[b * M + m] * vd;
}

template <int NQ, int LEVEL>
__global__ __attribute__((amdgpu_flat_work_group_size(1, ladder_threads<NQ>()))) void
ladder_kernel(const float* D, const float* geo, const float* q, float* rhs, Phys ph)
{
    constexpr int NF = kLadderFields;
    constexpr int NQ2 = NQ * NQ;
    constexpr int M = NQ * NQ2;
    __shared__ float sD[NQ2];
    __shared__ float sF[LEVEL >= 3 ? 2 * NF * NQ2 : 1];
    const int64_t e = blockIdx.x;
    const int t = threadIdx.x;
    const float* qe = q + e * (NF * M);
    const float* ge = geo + e * (10 * M);
    float* re = rhs + e * (NF * M);
    if constexpr (LEVEL >= 2) {
        for (int x = t; x < NQ2; x += ladder_threads<NQ>())
            sD[x] = D[x];
        __syncthreads();
    }
    const int i = t % NQ, j = t / NQ;
    const bool live = t < NQ2;
    for (int k = 0; k < NQ; ++k) {
        const int m = i + NQ * j + NQ2 * k;
        if constexpr (LEVEL <= 2) {
            if (live) {
                const float jinv = ge[9 * M + m];
                volatile float* vr = re + m;
                for (int d = 0; d < 2; ++d) {
                    const int row = d == 0 ? i : j;
                    for (int n = 0; n < NQ; ++n) {
                        const int mn = d == 0 ? n + NQ * j + NQ2 * k : i + NQ * n + NQ2 * k;
                        const float dn = LEVEL >= 2 ? sD[row * NQ + n] : D[row * NQ + n];
                        float F[NF];
                        ladder_flux<M>(qe, ge, mn, d, ph, F);
#pragma unroll
                        for (int b = 0; b < NF; ++b)
                            vr[b * M] = vr[b * M] - jinv * dn * F[b];
                    }
                }
            }
        } else {
            if (live) {
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    float F[NF];
                    ladder_flux<M>(qe, ge, m, d, ph, F);
#pragma unroll
                    for (int b = 0; b < NF; ++b)
                        sF[(d * NF + b) * NQ2 + i + NQ * j] = F[b];
                }
            }
            __syncthreads();
            if (live) {
                const float jinv = ge[9 * M + m];
                if constexpr (LEVEL == 3) {
                    volatile float* vr = re + m;
                    for (int d = 0; d < 2; ++d) {
                        const int row = d == 0 ? i : j;
                        for (int n = 0; n < NQ; ++n) {
                            const int ln = d == 0 ? n + NQ * j : i + NQ * n;
                            const float dn = sD[row * NQ + n];
#pragma unroll
                            for (int b = 0; b < NF; ++b)
                                vr[b * M] = vr[b * M] - jinv * dn * sF[(d * NF + b) * NQ2 + ln];
                        }
                    }
                } else {
                    float acc[NF];
#pragma unroll
                    for (int b = 0; b < NF; ++b)
                        acc[b] = 0.f;
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        const int row = d == 0 ? i : j;
#pragma unroll 2
                        for (int n = 0; n < NQ; ++n) {
                            const int ln = d == 0 ? n + NQ * j : i + NQ * n;
                            const float dn = LEVEL == 4 ? jinv * sD[row * NQ + n] : sD[row * NQ + n];
#pragma unroll
                            for (int b = 0; b < NF; ++b)
                                acc[b] += dn * sF[(d * NF + b) * NQ2 + ln];
                        }
                    }
#pragma unroll
                    for (int b = 0; b < NF; ++b)
                        re[b * M + m] -= LEVEL == 4 ? acc[b] : jinv * acc[b];
                }
            }
            __syncthreads();   // sF is rewritten by the next slice
        }
    }
}

}  // namespace semk

namespace semh {

template <int NQ, int LEVEL>
static hipError_t ladder_one(int64_t Ne, const float* D, const float* geo, const float* q,
                             float* rhs, const semk::Phys& ph, hipStream_t s)
{
    if (!dispatch_fits(Ne, semk::ladder_threads<NQ>()))
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((semk::ladder_kernel<NQ, LEVEL>), dim3((unsigned)Ne),
                       dim3(semk::ladder_threads<NQ>()), 0, s, D, geo, q, rhs, ph);
    return hipGetLastError();
}

bool ladder_supported(int nq)
{
#define SEM_X(NQ_)  \
    if (nq == NQ_)  \
        return true;
    SEM_LADDER_NQ(SEM_X)
#undef SEM_X
    return false;
}

hipError_t launch_ladder(int level, int nq, int64_t Ne, const float* D, const float* geo,
                         const float* q, float* rhs, const semk::Phys& ph, hipStream_t s)
{
#define SEM_X(NQ_)                                                                  \
    if (nq == NQ_) {                                                                \
        switch (level) {                                                            \
        case 1: return ladder_one<NQ_, 1>(Ne, D, geo, q, rhs, ph, s);               \
        case 2: return ladder_one<NQ_, 2>(Ne, D, geo, q, rhs, ph, s);               \
        case 3: return ladder_one<NQ_, 3>(Ne, D, geo, q, rhs, ph, s);               \
        case 4: return ladder_one<NQ_, 4>(Ne, D, geo, q, rhs, ph, s);               \
        case 5: return ladder_one<NQ_, 5>(Ne, D, geo, q, rhs, ph, s);               \
        default: return hipErrorInvalidValue;                                       \
        }                                                                           \
    }
    SEM_LADDER_NQ(SEM_X)
#undef SEM_X
    return hipErrorInvalidValue;
}

}  // namespace semh
