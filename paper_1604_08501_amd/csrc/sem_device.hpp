// Device-side building blocks of the strong-form volume term (Sec. 2,
// Eq. (volterm)) for gfx950.  Everything here is internal to libsem.so.
//
// Layouts (element outermost, structure-of-arrays inside an element):
//   q, rhs, lambda, mu : [Ne][5][Nq^3]   fields rho, U1, U2, U3, Theta
//   geo                : [Ne][10][Nq^3]  slot 3*d + a = g_{a d}, slot 9 = 1/J
//   rho_ref            : [Ne][Nq^3]      (same dtype as q)
//   theta_ref          : [Ne][Nq^3]      always FP64
//   D                  : [Nq][Nq]        D[i*Nq + n] = l_n'(xi_i)
//   node m = i + Nq*j + Nq^2*k, with i, j, k along r, s, t (Fig. 1).
//
// One workgroup owns a tile of EPB whole elements.  Every thread handles
// the nodes tid, tid + NT, ... of the tile.  Phase 1 reads each node's state
// and metric terms once, evaluates the pressure and the contravariant fluxes
// of all three reference directions and stages them in LDS (the paper's
// flux precompute and state prefetch); phase 2 applies D along r, s and t
// out of LDS, accumulates in registers, applies 1/J once (distributive
// law), adds the gravity source and writes each output once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace semk {

struct Phys {
    double p0, gamma, R, grav;
    double r_over_p0;   // R / p0, formed once on the host
};

template <typename T>
struct BlockPtrs {
    const T* D;
    const T* geo;
    const T* q;
    const T* rho_ref;        // nullable (then rho_ref = 0)
    const double* theta_ref; // nullable (then the full pressure is used)
    T* rhs;
    int64_t Ne;
    const T* rk_x;           // fused Runge-Kutta stage only: x of out = a x + b (q + dt v)
};

// Arrays of the surface term (face term of dq/dt = v + s).
template <typename T>
struct SurfPtrs {
    const int32_t* nbr;         // [Ne][6] element across faces r-, r+, s-, s+, t-, t+
    const T* geo;               // [Ne][10][M]
    const T* q;                 // [Ne][5][M]
    const double* theta_ref;    // [Ne][M] or null
    T* rhs;                     // [Ne][5][M]
    int64_t Ne;
};

// Stage update of an explicit Runge-Kutta method fused into the epilogue of
// the volume term: out = a*x + b*(q + dt*v(q)), x not read when a == 0.
struct RkStage {
    double a, b, dt;
};

// Device-side descriptor of one block of a mixed-order batch launch: its
// arrays, the physical constants and the fused stage coefficients.
template <typename T>
struct BatchBlock {
    BlockPtrs<T> b;
    Phys ph;
    RkStage rk;
};

// Streaming accesses: every per-node input of a launch is read once and every
// output written once, so they carry the nontemporal hint and do not displace
// cache lines that are reused (D, per-element metric records).  At N = 7 this
// measured 6% (FP64) and 12% (FP32) faster than cached accesses.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p)
{
    return __builtin_nontemporal_load(p);
}

template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// 1/x: the FP64 quotient; in FP32 the hardware reciprocal (1 ulp), which
// spares the 10-instruction IEEE division sequence and its denormal-mode
// switches (the FP32 volume + surface launch 12% faster; results within a
// few 1e-7 of the divided ones)
template <typename T>
__device__ __forceinline__ T recip(T x)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_amdgcn_rcpf(x);
    else
        return (T)1 / x;
}

// sqrt: FP64 correctly rounded; in FP32 the hardware square root (1 ulp),
// used for the sound speeds and normal lengths of the face terms
template <typename T>
__device__ __forceinline__ T root(T x)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_amdgcn_sqrtf(x);
    else
        return sqrt(x);
}

// ---------------------------------------------------------------------------
// Pressure entering the flux (Sec. 2 EOS p = p0 (R Theta / p0)^gamma).
// With a reference state it is the perturbation p - p_ref.
// ---------------------------------------------------------------------------
template <typename T>
struct Pressure;

template <>
struct Pressure<double> {
    // FP64: x^gamma as exp(gamma log x) with the library log and exp.  For
    // the states of an atmosphere (x = R Theta / p0 of order one) the error of
    // gamma*log(x) is a few ulp of a number of order 0.1, so the result keeps
    // full FP64 accuracy while costing far less than a general pow.  The two
    // powers are differenced before the scaling by p0, so that
    // Theta == Theta_ref gives exactly zero.
    static __device__ __forceinline__ double xgamma(double x, const Phys& ph)
    {
        return exp(ph.gamma * log_pos(x));
    }
    // log x from the mathematics: x = 2^e m with m in [sqrt(1/2), sqrt(2)),
    // log x = e ln 2 + 2 atanh(s) with s = (m - 1)/(m + 1), |s| <= 0.1716, and
    // 2 atanh(s) = 2s + 2s z (1/3 + z/5 + ... + z^8/19), z = s^2, the Taylor
    // series cut where the next term is below 2^-55 of the sum, evaluated by
    // Estrin's scheme (four dependent steps instead of Horner's eight: the
    // k-slice tile at Nq = 12, where the pressure sits between a workgroup's
    // loads and its barrier, ran 25% slower with Horner's).  m - 1 is
    // exact, so s carries the roundings of one sum and one quotient; ln 2
    // enters as a two-part constant, so e ln 2 adds no rounding of its own.
    // The hardware frexp also splits subnormals; zero gives -inf, negative
    // arguments and NaN give NaN and +inf gives +inf, as the library log.
    // A third of the instructions of the library log.
    static __device__ __forceinline__ double log_pos(double x)
    {
        double m = __builtin_amdgcn_frexp_mant(x);   // [1/2, 1)
        int e = __builtin_amdgcn_frexp_exp(x);
        if (m < 0x1.6a09e667f3bcdp-1) {
            m *= 2.0;
            e -= 1;
        }
        const double s = (m - 1.0) / (m + 1.0);
        const double z = s * s;
        const double z2 = z * z, z4 = z2 * z2;
        const double p01 = fma(1.0 / 5.0, z, 1.0 / 3.0), p23 = fma(1.0 / 9.0, z, 1.0 / 7.0);
        const double p45 = fma(1.0 / 13.0, z, 1.0 / 11.0), p67 = fma(1.0 / 17.0, z, 1.0 / 15.0);
        const double p03 = fma(p23, z2, p01), p47 = fma(p67, z2, p45);
        const double q = fma(fma(1.0 / 19.0, z4, p47), z4, p03);
        const double s2 = 2.0 * s;
        const double lm = fma(s2 * z, q, s2);
        constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;    // ln 2 rounded to double
        constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;   // ln 2 - kLn2Hi
        const double ed = (double)e;
        const double r = fma(ed, kLn2Hi, fma(ed, kLn2Lo, lm));
        if (x > 0.0 && x < __builtin_inf())
            return r;
        return x == 0.0 ? -__builtin_inf() : (x > 0.0 ? x : __builtin_nan(""));
    }
    static __device__ __forceinline__ double eval(double Th, bool has_ref, double thr,
                                                  const Phys& ph)
    {
        const double s = ph.r_over_p0;
        double x = xgamma(s * Th, ph);
        if (has_ref)
            x -= xgamma(s * thr, ph);
        return ph.p0 * x;
    }
    // the flux pressure of eval() and the full pressure p (for the sound
    // speed of the surface term's dissipation)
    static __device__ __forceinline__ void eval_full(double Th, bool has_ref, double thr,
                                                     const Phys& ph, double& pflux, double& pfull)
    {
        const double s = ph.r_over_p0;
        const double x = xgamma(s * Th, ph);
        pfull = ph.p0 * x;
        pflux = has_ref ? ph.p0 * (x - xgamma(s * thr, ph)) : pfull;
    }
    // dp/dTheta = gamma p / Theta (full pressure, for the adjoint)
    static __device__ __forceinline__ double dp_dtheta(double Th, const Phys& ph)
    {
        return ph.gamma * (ph.p0 * xgamma(ph.r_over_p0 * Th, ph)) / Th;
    }
};

template <>
struct Pressure<float> {
    // FP32 perturbation form: Theta' = Theta - Theta_ref is formed in FP64
    // (Theta_ref is stored in FP64), then
    //   p' = p_ref * expm1(gamma * log1p(Theta'/Theta_ref)),
    // which uses EOS(Theta)/EOS(Theta_ref) = (Theta/Theta_ref)^gamma and keeps
    // the relative accuracy of the small perturbation instead of cancelling
    // two large FP32 pressures.
    // x^gamma = 2^(gamma log2 x) with the hardware log2 and exp2 (about 1 ulp
    // each) for positive normal x: at most 1.4e-6 relative error over
    // [1e-3, 1e3] against FP64 pow (the library expf(gamma logf(x)): 2.1e-6),
    // in three instructions
    static __device__ __forceinline__ float xgamma(float x, float g)
    {
        return __builtin_amdgcn_exp2f(g * __builtin_amdgcn_logf(x));
    }
    // log(1 + x) by Goldberg's method (Theorem 4 of "What every computer
    // scientist should know about floating-point arithmetic", 1991): with
    // u = 1 + x rounded, log(1 + x) = x if u == 1, else log(u) x / (u - 1).
    // The factor x / (u - 1) undoes the rounding of u, so small x keeps its
    // digits; with the hardware log2 (times ln 2) and reciprocal the relative
    // error stays a few ulp (at most 4.2 over 7.3e7 arguments in [-0.5, 1]).
    // It costs a log and a reciprocal, a small part of the instructions of
    // the library log1pf.
    static __device__ __forceinline__ float log1p_g(float x)
    {
        const float u = 1.0f + x;
        return u == 1.0f ? x
                         : (__builtin_amdgcn_logf(u) * 0x1.62e430p-1f) *
                               (x * __builtin_amdgcn_rcpf(u - 1.0f));
    }
    static __device__ __forceinline__ float eval(float Th, bool has_ref, double thr,
                                                 const Phys& ph)
    {
        const float p0 = (float)ph.p0, g = (float)ph.gamma, s = (float)ph.r_over_p0;
        if (has_ref) {
            const float dth = (float)((double)Th - thr);
            const float trf = (float)thr;
            const float pref = p0 * xgamma(s * trf, g);
            return pref * expm1f(g * log1p_g(dth * __builtin_amdgcn_rcpf(trf)));
        }
        return p0 * xgamma(s * Th, g);
    }
    static __device__ __forceinline__ float dp_dtheta(float Th, const Phys& ph)
    {
        const float p0 = (float)ph.p0, g = (float)ph.gamma, s = (float)ph.r_over_p0;
        return g * (p0 * xgamma(s * Th, g)) / Th;
    }
    // eval() and the full pressure p_ref + p' (or p)
    static __device__ __forceinline__ void eval_full(float Th, bool has_ref, double thr,
                                                     const Phys& ph, float& pflux, float& pfull)
    {
        const float p0 = (float)ph.p0, g = (float)ph.gamma, s = (float)ph.r_over_p0;
        if (has_ref) {
            const float dth = (float)((double)Th - thr);
            const float trf = (float)thr;
            const float pref = p0 * xgamma(s * trf, g);
            pflux = pref * expm1f(g * log1p_g(dth * __builtin_amdgcn_rcpf(trf)));
            pfull = pref + pflux;
        } else {
            pfull = pflux = p0 * xgamma(s * Th, g);
        }
    }
};

template <int NQ>
struct Shape {
    static constexpr int NQ2 = NQ * NQ;
    static constexpr int M = NQ * NQ * NQ;
    // D is staged in front of the flux area; pad it to 16 bytes
    template <typename T>
    static constexpr int d_slots()
    {
        return ((NQ2 * (int)sizeof(T) + 15) / 16) * 16 / (int)sizeof(T);
    }
};

// Tile layouts.  FULL keeps the contravariant fluxes of every active
// direction of every node in LDS (one barrier); ALIAS keeps one direction at
// a time and walks the directions in separate LDS phases, trading barriers
// for a fraction of the LDS, which lets large elements (Nq >= 9) and the
// worst-case shape of a mixed-order batch keep more workgroups resident.
enum Layout : int { FULL = 0, ALIAS = 1 };

// Fields per node: NF = 5 (rho, U1, U2, U3, Theta) or 8 (plus the passive
// tracers Q1..Q3, whose flux is U_a Q_i / rho).  Active reference directions:
// bit 0 r, bit 1 s, bit 2 t (DIRS = 7 for the full volume term, 3 for the
// paper's fused r+s benchmark kernel).
template <int DIRS>
constexpr int ndirs()
{
    return ((DIRS & 1) != 0) + ((DIRS & 2) != 0) + ((DIRS & 4) != 0);
}

// position of direction d among the active ones (its LDS slot in FULL tiles)
template <int DIRS>
constexpr int dir_slot(int d)
{
    int s = 0;
    for (int x = 0; x < d; ++x)
        s += (DIRS >> x) & 1;
    return s;
}

template <int NQ, int EPB, int NT>
constexpr int nodes_per_thread()
{
    return (EPB * Shape<NQ>::M + NT - 1) / NT;
}

// ALIAS tiles keep each node's state in registers: at most 2 nodes per thread
// in FP64, 4 in FP32.
template <typename T>
constexpr int alias_max_nodes_per_thread()
{
    return sizeof(T) == 4 ? 4 : 2;
}

// A thread of a FULL tile that handles more than one node keeps 1/J and the
// gravity source of its nodes in LDS (two extra values per node) instead of
// register arrays, so that its node loop need not be unrolled.
// The r contraction runs in registers, with the r line's fluxes exchanged
// between the lanes of a wave (DPP lane permutations), when an r line is 2, 4
// or 8 adjacent lanes (Nq = 2, 4, 8; node m = i + Nq j + ... sits in lane
// m mod 64) and the tile keeps each node's partial sums in registers (ALIAS,
// or FULL with one node per thread).  Its fluxes then never touch LDS.
constexpr bool kRegisterR = true;

template <int NQ, int EPB, int NT, int LAY, int DIRS>
constexpr bool r_in_registers()
{
    return kRegisterR && (DIRS & 1) != 0 && (NQ == 2 || NQ == 4 || NQ == 8) &&
           (LAY == ALIAS || nodes_per_thread<NQ, EPB, NT>() == 1);
}

// Directions whose fluxes a tile stages in LDS.
template <int NQ, int EPB, int NT, int LAY, int DIRS>
constexpr int lds_dirs()
{
    return r_in_registers<NQ, EPB, NT, LAY, DIRS>() ? (DIRS & ~1) : DIRS;
}

template <typename T, int NQ, int EPB, int NT, int LAY, int NF = 5, int DIRS = 7>
constexpr int volume_tile_values_per_node()
{
    if (LAY == ALIAS)
        return NF;
    return ndirs<lds_dirs<NQ, EPB, NT, LAY, DIRS>()>() * NF +
           (nodes_per_thread<NQ, EPB, NT>() > 1 ? 2 : 0);
}

// LDS bytes a forward tile needs: D plus the staged values of every node.
template <typename T, int NQ, int EPB, int NT, int LAY, int NF = 5, int DIRS = 7>
constexpr int volume_tile_lds_bytes()
{
    return (Shape<NQ>::template d_slots<T>() +
            EPB * volume_tile_values_per_node<T, NQ, EPB, NT, LAY, NF, DIRS>() * Shape<NQ>::M) *
           (int)sizeof(T);
}

// The stage input q of the fused Runge-Kutta epilogue, taken from the node's
// state when it is read.  The other epilogue input, x (when a != 0), is read
// at the store: reading it with the state kept 5 more values per node live
// through the tile, which pushed the two-node aliased shapes past the
// register budget into scratch spills (FP64 RK3 step 0.969 -> 0.935 ms,
// FP32 0.512 -> 0.500 ms without them).
template <typename T, bool RK>
struct RkNode {
    template <typename S>
    __device__ __forceinline__ void load(const BlockPtrs<T>&, const RkStage&, int64_t, int, int,
                                         const S&)
    {
    }
};

template <typename T>
struct RkNode<T, true> {
    T q[5];
    template <typename S>
    __device__ __forceinline__ void load(const BlockPtrs<T>&, const RkStage&, int64_t, int, int,
                                         const S& st)
    {
        q[0] = st.rho;
        q[1] = st.U1;
        q[2] = st.U2;
        q[3] = st.U3;
        q[4] = st.Th;
    }
};

// Epilogue for one node: rhs = -(1/J) acc + source (+ rhs when ACC), or the
// fused Runge-Kutta stage out = a x + b (q + dt v) when RK (five fields).
template <typename T, int M, int NF, bool ACC, bool RK, bool STREAM = true>
__device__ __forceinline__ void store_node(const BlockPtrs<T>& B, const RkStage& rk, int64_t e,
                                           int m, const T (&acc)[NF], T jinv, T src,
                                           const RkNode<T, RK>& rn)
{
    static_assert(!RK || NF == 5, "the fused Runge-Kutta stage is for the five-field state");
    T* __restrict__ re = B.rhs + e * (NF * M) + m;
    T x[RK ? 5 : 1];
    if constexpr (RK) {
        const T* xe = B.rk_x + e * (5 * M) + m;
#pragma unroll
        for (int b = 0; b < 5; ++b)
            x[b] = rk.a != 0.0 ? ld_stream(xe + b * M) : (T)0;
    }
#pragma unroll
    for (int b = 0; b < NF; ++b) {
        T v = -jinv * acc[b];
        if (b == 3)
            v += src;
        if constexpr (RK) {
            st_stream(re + b * M, (T)rk.a * x[b] + (T)rk.b * (rn.q[b] + (T)rk.dt * v));
        } else if constexpr (STREAM) {
            if constexpr (ACC)
                v += ld_stream(re + b * M);
            st_stream(re + b * M, v);
        } else {
            if constexpr (ACC)
                v += re[b * M];
            re[b * M] = v;
        }
    }
}

// Pointwise part for one node: pressure (perturbation when a reference is
// given), 1/rho, metric terms of the active directions, 1/J, the gravity
// source and the tracers.
template <typename T, int NF>
struct NodeState {
    T rho, U1, U2, U3, Th, rinv, pp, jinv, src;
    T pfull;   // full pressure (FULLP loads only)
    T g[9];
    T Q[NF > 5 ? NF - 5 : 1];
};

// GEOE: the metric terms are given once per element (affine elements,
// geo[e][10]) instead of at every node (geo[e][10][Nq^3]).  STREAM = false
// reads through the cache (for tiles whose consecutive accesses share cache
// lines).  SRC = false leaves the gravity source out (src = 0, rho_ref not
// read), for a pass that adds one direction's term to a finished rhs.
// FULLP = true also keeps the full pressure (for the surface term) and reads
// the state and Theta_ref through the cache: the face neighbours of the
// element read its face values again.
template <typename T, int M, int NF, int DIRS, bool GEOE = false, bool STREAM = true,
          bool SRC = true, bool FULLP = false>
__device__ __forceinline__ void load_node(const BlockPtrs<T>& B, const Phys& ph, int64_t e, int m,
                                          NodeState<T, NF>& st)
{
    const T* __restrict__ qe = B.q + e * (NF * M) + m;
    constexpr int GS = GEOE ? 1 : M;   // stride between metric slots
    const T* __restrict__ ge = GEOE ? B.geo + e * 10 : B.geo + e * (10 * M) + m;
    // per-element metric records are shared by every node of the element and
    // stay cached; everything else streams
    auto ld = [](const auto* p) { return STREAM ? ld_stream(p) : *p; };
    auto ldq = [](const auto* p) { return (STREAM && !FULLP) ? ld_stream(p) : *p; };
    auto geo_at = [&](int s) { return GEOE ? ge[s * GS] : ld(ge + s * GS); };
    const T rho = ldq(qe);
    st.rho = rho;
    st.U1 = ldq(qe + M);
    st.U2 = ldq(qe + 2 * M);
    st.U3 = ldq(qe + 3 * M);
    st.Th = ldq(qe + 4 * M);
#pragma unroll
    for (int b = 5; b < NF; ++b)
        st.Q[b - 5] = ldq(qe + b * M);
#pragma unroll
    for (int s = 0; s < 9; ++s)
        st.g[s] = ((DIRS >> (s / 3)) & 1) ? geo_at(s) : (T)0;
    st.jinv = geo_at(9);
    const bool has_ref = B.theta_ref != nullptr;
    T rr = (T)0;
    double thr = 0.0;
    if (has_ref) {
        if constexpr (SRC)
            rr = ld(B.rho_ref + e * M + m);
        thr = ldq(B.theta_ref + e * M + m);
    }
    st.src = SRC ? -(T)ph.grav * (rho - rr) : (T)0;
    if constexpr (FULLP)
        Pressure<T>::eval_full(st.Th, has_ref, thr, ph, st.pp, st.pfull);
    else
        st.pp = Pressure<T>::eval(st.Th, has_ref, thr, ph);
    st.rinv = recip(rho);
}

// Contravariant flux of direction d (sum_a g_ad f_a) of one node into LDS:
// F[b*M] for the fields b = rho, U1, U2, U3, Theta (and the tracers).
template <typename T, int M, int NF>
__device__ __forceinline__ void put_flux(const NodeState<T, NF>& st, int d, T* __restrict__ F)
{
    const T g1 = st.g[3 * d], g2 = st.g[3 * d + 1], g3 = st.g[3 * d + 2];
    const T Ud = g1 * st.U1 + g2 * st.U2 + g3 * st.U3;   // contravariant momentum
    const T vd = Ud * st.rinv;
    F[0] = Ud;
    F[M] = st.U1 * vd + g1 * st.pp;
    F[2 * M] = st.U2 * vd + g2 * st.pp;
    F[3 * M] = st.U3 * vd + g3 * st.pp;
    F[4 * M] = st.Th * vd;
#pragma unroll
    for (int b = 5; b < NF; ++b)
        F[b * M] = st.Q[b - 5] * vd;
}

// acc[b] += sum_n D[row][n] F_b(base + n*stride), b < NF, out of LDS.
// UNR: unroll factor of the n loop (2 by default: full unrolling hoists every
// LDS load and spills in tiles holding several nodes per thread).
template <typename T, int NQ, int M, int NF, int UNR = 2>
__device__ __forceinline__ void contract(const T* __restrict__ sD, const T* __restrict__ F, int row,
                                         int stride, T (&acc)[NF])
{
#pragma unroll UNR
    for (int n = 0; n < NQ; ++n) {
        const T dn = sD[row * NQ + n];
#pragma unroll
        for (int b = 0; b < NF; ++b)
            acc[b] += dn * F[b * M + n * stride];
    }
}

// D along direction d for the node (i, j, k): r runs over i (stride 1),
// s over j (stride Nq), t over k (stride Nq^2).
template <typename T, int NQ, int M, int NF, int UNR = 2>
__device__ __forceinline__ void contract_dir(const T* __restrict__ sD, const T* __restrict__ Fd,
                                             int d, int i, int j, int k, T (&acc)[NF])
{
    constexpr int NQ2 = NQ * NQ;
    if (d == 0)
        contract<T, NQ, M, NF, UNR>(sD, Fd + NQ * j + NQ2 * k, i, 1, acc);
    else if (d == 1)
        contract<T, NQ, M, NF, UNR>(sD, Fd + i + NQ2 * k, j, NQ, acc);
    else
        contract<T, NQ, M, NF, UNR>(sD, Fd + i + NQ * j, k, NQ2, acc);
}

// Value of lane (this lane with its index bits permuted by CTRL) within the
// same row of 16 lanes: CTRL is a DPP control (quad_perm or row_half_mirror).
// 64-bit values move as two 32-bit halves.
template <int CTRL, typename T>
__device__ __forceinline__ T lane_perm(T v)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(
            T, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
    } else {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, false);
        const unsigned hi =
            (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
        return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    }
}

constexpr int kQuadXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kQuadXor3 = 0x1B;        // quad_perm [3, 2, 1, 0]
constexpr int kHalfRowMirror = 0x141;  // lane l of 8 <- lane 7 - l = l ^ 7

// acc[b] += sum_n D[i][n] F_b(n) along an r line held one node per lane
// (lanes i = 0..NQ-1 of an aligned group): lane i ^ x for x = 0..NQ-1 are
// visited with quad permutations (x = 1, 2, 3) and the half-row mirror
// (x = 7, then 6, 5, 4).  f holds this lane's own fluxes.
template <typename T, int NQ, int NF>
__device__ __forceinline__ void contract_r_lanes(const T* __restrict__ sD, const T (&f)[NF], int i,
                                                 T (&acc)[NF])
{
    static_assert(NQ == 2 || NQ == 4 || NQ == 8, "r lines of 2, 4 or 8 lanes");
    const T* __restrict__ Di = sD + i * NQ;
    auto add = [&](const T (&g)[NF], int x) {
        const T dn = Di[i ^ x];
#pragma unroll
        for (int b = 0; b < NF; ++b)
            acc[b] += dn * g[b];
    };
    auto perm = [&](const T (&src)[NF], T (&dst)[NF], auto ctrl) {
#pragma unroll
        for (int b = 0; b < NF; ++b)
            dst[b] = lane_perm<decltype(ctrl)::value>(src[b]);
    };
    T g[NF];
    add(f, 0);
    perm(f, g, std::integral_constant<int, kQuadXor1>{});
    add(g, 1);
    if constexpr (NQ >= 4) {
        perm(f, g, std::integral_constant<int, kQuadXor2>{});
        add(g, 2);
        perm(f, g, std::integral_constant<int, kQuadXor3>{});
        add(g, 3);
    }
    if constexpr (NQ == 8) {
        T h[NF];
        perm(f, h, std::integral_constant<int, kHalfRowMirror>{});
        add(h, 7);
        perm(h, g, std::integral_constant<int, kQuadXor1>{});
        add(g, 6);
        perm(h, g, std::integral_constant<int, kQuadXor2>{});
        add(g, 5);
        perm(h, g, std::integral_constant<int, kQuadXor3>{});
        add(g, 4);
    }
}

// ---------------------------------------------------------------------------
// Surface term of dq/dt = v + s fused into the forward tile's epilogue (the
// strong-form discontinuous Galerkin face term with a local Lax-Friedrichs
// flux; see the surface kernel for the formula).  Faces f = 2 d + side of an
// element; a face node is named by its indices (a2, b2) along the face's two
// tangential directions (for d = r: s, t; for s: r, t; for t: r, s), and
// meets the node with the same tangential indices at the other end of
// direction d in the element across the face.
// ---------------------------------------------------------------------------

// Workgroup index whose elements this workgroup handles: hardware workgroup
// b runs on accelerator complex die (XCD) b mod 8 of MI355X; the first
// 8 floor(G/8) workgroups are re-dealt so that XCD x handles logical
// workgroups [x G8/8, (x+1) G8/8) in order, which keeps an element and its
// neighbours along r and s on one XCD's L2 at about the same time.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_contiguous_block(int64_t b, int64_t G)
{
    const int64_t G8 = (G / kXcds) * kXcds;
    if (b >= G8)
        return b;
    const int64_t per = G8 / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

// Values staged per neighbour face node: the state (5), the flux pressure
// and the sound speed sqrt(gamma p / rho) of the full pressure.
constexpr int kFaceVals = 7;

// Values staged per own face node by its owner: the state (5), the flux
// pressure, the sound speed, the outward normal times its area factor (3)
// and 1/rho.
constexpr int kOwnVals = 11;

template <int NQ>
constexpr int face_lds_values_per_element()
{
    return 6 * (kFaceVals + kOwnVals) * NQ * NQ;
}

// Node of face (d, side) with tangential indices (a2, b2).
template <int NQ>
__device__ __forceinline__ int face_node(int d, int side, int a2, int b2)
{
    const int sd = d == 0 ? 1 : (d == 1 ? NQ : NQ * NQ);
    const int sa = d == 0 ? NQ : 1;
    const int sb = d == 2 ? NQ : NQ * NQ;
    return (side ? NQ - 1 : 0) * sd + a2 * sa + b2 * sb;
}

// The tile's neighbour face values into LDS, sF[es][f][v][a2 + NQ b2]: for
// face f of tile element es, the state of the element across f at its node
// facing ours, its flux pressure and its sound speed.  Faces whose neighbour
// index lies outside [0, Ne) are boundary faces: nothing is read.
template <typename T, int NQ, int EPB, int NT>
__device__ __forceinline__ void stage_neighbour_faces(const BlockPtrs<T>& B,
                                                      const int32_t* __restrict__ nbr,
                                                      const Phys& ph, int64_t e0, int ne,
                                                      T* __restrict__ sFace)
{
    constexpr int NQ2 = NQ * NQ;
    constexpr int M = NQ2 * NQ;
    constexpr int PER = 6 * NQ2;
    const bool has_ref = B.theta_ref != nullptr;
    const T gam = (T)ph.gamma;
#pragma unroll 1
    for (int x = threadIdx.x; x < EPB * PER; x += NT) {
        const int es = x / PER;
        const int r = x - es * PER;
        const int f = r / NQ2;
        const int a = r - f * NQ2;
        if (es >= ne)
            continue;
        const int64_t en = nbr[(e0 + es) * 6 + f];
        if (en < 0 || en >= B.Ne)
            continue;
        const int d = f >> 1, side = f & 1;
        const int mp = face_node<NQ>(d, 1 - side, a % NQ, a / NQ);
        const T* __restrict__ qn = B.q + en * (5 * M) + mp;
        T v[kFaceVals];
#pragma unroll
        for (int b = 0; b < 5; ++b)
            v[b] = qn[b * M];
        const double thr = has_ref ? B.theta_ref[en * M + mp] : 0.0;
        T pfull;
        Pressure<T>::eval_full(v[4], has_ref, thr, ph, v[5], pfull);
        v[6] = root(gam * pfull / v[0]);
        T* __restrict__ o = sFace + es * (kFaceVals * PER) + f * (kFaceVals * NQ2) + a;
#pragma unroll
        for (int b = 0; b < kFaceVals; ++b)
            o[b * NQ2] = v[b];
    }
}

// The owner of a boundary node stages, for each face of the element the node
// lies on, the node's state, flux pressure, sound speed, outward normal N
// (sigma (g_0d, g_1d, g_2d) at the node) and 1/rho in sOwn[f][v][a].
template <typename T, int NQ>
__device__ __forceinline__ void stage_own_faces(const NodeState<T, 5>& st, int i, int j, int k,
                                                T gam, T* __restrict__ sOwn)
{
    constexpr int NQ2 = NQ * NQ;
    constexpr int N = NQ - 1;
    const int ijk[3] = {i, j, k};
    if (!(i == 0 || i == N || j == 0 || j == N || k == 0 || k == N))
        return;
    const T c = root(gam * st.pfull * st.rinv);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int id = ijk[d];
        if (id != 0 && id != N)
            continue;
        const int side = id == N ? 1 : 0;
        const int a = d == 0 ? j + NQ * k : (d == 1 ? i + NQ * k : i + NQ * j);
        const T sg = side ? (T)1 : (T)-1;
        const T v[kOwnVals] = {st.rho, st.U1, st.U2, st.U3, st.Th, st.pp, c,
                               sg * st.g[3 * d], sg * st.g[3 * d + 1], sg * st.g[3 * d + 2],
                               st.rinv};
        T* __restrict__ o = sOwn + (2 * d + side) * (kOwnVals * NQ2) + a;
#pragma unroll
        for (int b = 0; b < kOwnVals; ++b)
            o[b * NQ2] = v[b];
    }
}

// One thread per face node of the tile: F* - Fn(q-) of the five fields from
// the staged own and neighbour values, written over the neighbour's state in
// sFace (zero for a boundary face).
template <typename T, int NQ, int EPB, int NT>
__device__ __forceinline__ void face_fluxes(const int32_t* __restrict__ nbr, int64_t Ne, int64_t e0,
                                            int ne, T* __restrict__ sFace,
                                            const T* __restrict__ sOwn)
{
    constexpr int NQ2 = NQ * NQ;
    constexpr int PER = 6 * NQ2;
#pragma unroll 1
    for (int x = threadIdx.x; x < EPB * PER; x += NT) {
        const int es = x / PER;
        const int r = x - es * PER;
        const int f = r / NQ2;
        const int a = r - f * NQ2;
        if (es >= ne)
            continue;
        T* __restrict__ v = sFace + es * (kFaceVals * PER) + f * (kFaceVals * NQ2) + a;
        const int64_t en = nbr[(e0 + es) * 6 + f];
        if (en < 0 || en >= Ne) {
#pragma unroll
            for (int b = 0; b < 5; ++b)
                v[b * NQ2] = (T)0;   // boundary face: exterior state = interior state
            continue;
        }
        const T* __restrict__ o = sOwn + es * (kOwnVals * PER) + f * (kOwnVals * NQ2) + a;
        T qm[5], qp[5];
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            qm[b] = o[b * NQ2];
            qp[b] = v[b * NQ2];
        }
        const T pm = o[5 * NQ2], cm = o[6 * NQ2];
        const T n0 = o[7 * NQ2], n1 = o[8 * NQ2], n2 = o[9 * NQ2], rinv_m = o[10 * NQ2];
        const T pp = v[5 * NQ2], cp = v[6 * NQ2];
        const T nn = root(n0 * n0 + n1 * n1 + n2 * n2);
        const T rinv_p = recip(qp[0]);
        const T NUm = n0 * qm[1] + n1 * qm[2] + n2 * qm[3];
        const T NUp = n0 * qp[1] + n1 * qp[2] + n2 * qp[3];
        const T vm = NUm * rinv_m, vp = NUp * rinv_p;   // N . u on each side
        const T inn = recip(nn);
        const T lam_m = fabs(vm) * inn + cm;
        const T lam_p = fabs(vp) * inn + cp;
        const T diss = (T)0.5 * (lam_m > lam_p ? lam_m : lam_p) * nn;
        const T dp = pp - pm;
        const T dF[5] = {NUp - NUm, qp[1] * vp - qm[1] * vm + n0 * dp,
                         qp[2] * vp - qm[2] * vm + n1 * dp, qp[3] * vp - qm[3] * vm + n2 * dp,
                         qp[4] * vp - qm[4] * vm};
#pragma unroll
        for (int b = 0; b < 5; ++b)
            v[b * NQ2] = (T)0.5 * dF[b] - diss * (qp[b] - qm[b]);
    }
}

// acc[b] += (1/w_N) sum over the node's faces of (F* - Fn(q-))_b, so that the
// epilogue's -(1/J) acc + source is v + s; faces visited r, s, t in order.
// sFe: the element's face results, VALS values per face node slot.
template <typename T, int NQ, int VALS = kFaceVals>
__device__ __forceinline__ void gather_face_terms(int i, int j, int k,
                                                  const T* __restrict__ sFe, T lift, T (&acc)[5])
{
    constexpr int NQ2 = NQ * NQ;
    constexpr int N = NQ - 1;
    const int ijk[3] = {i, j, k};
    if (!(i == 0 || i == N || j == 0 || j == N || k == 0 || k == N))
        return;
    T sacc[5] = {(T)0, (T)0, (T)0, (T)0, (T)0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int id = ijk[d];
        if (id != 0 && id != N)
            continue;
        const int side = id == N ? 1 : 0;
        const int a = d == 0 ? j + NQ * k : (d == 1 ? i + NQ * k : i + NQ * j);
        const T* __restrict__ v = sFe + (2 * d + side) * (VALS * NQ2) + a;
#pragma unroll
        for (int b = 0; b < 5; ++b)
            sacc[b] += v[b * NQ2];
    }
#pragma unroll
    for (int b = 0; b < 5; ++b)
        acc[b] += lift * sacc[b];
}

// Inputs of the fused surface term: the neighbour table, 1/w_N, and the
// LDS of the staged neighbour faces.
template <typename T>
struct SurfIn {
    const int32_t* nbr;
    T lift;
    T* sFace;   // [EPB][6][kFaceVals][Nq^2]: neighbour values, then F* - Fn(q-)
    T* sOwn;    // [EPB][6][kOwnVals][Nq^2]: the element's own face values
};

// ---------------------------------------------------------------------------
// Forward tile: EPB elements starting at e0, of which the first ne exist.
// ---------------------------------------------------------------------------
template <typename T, int NQ, int EPB, int NT, bool ACC, bool RK, int NF, int DIRS, bool GEOE,
          int UNR = 2>
__device__ __forceinline__ void volume_tile_full(const BlockPtrs<T>& B, int64_t e0, int ne,
                                                 const Phys& ph, const RkStage& rk,
                                                 T* __restrict__ smem)
{
    constexpr int NQ2 = Shape<NQ>::NQ2;
    constexpr int M = Shape<NQ>::M;
    constexpr int NODES = EPB * M;
    constexpr int NPT = nodes_per_thread<NQ, EPB, NT>();
    constexpr int VPN = volume_tile_values_per_node<T, NQ, EPB, NT, FULL, NF, DIRS>();
    constexpr bool RREG = r_in_registers<NQ, EPB, NT, FULL, DIRS>();
    constexpr int LD = lds_dirs<NQ, EPB, NT, FULL, DIRS>();   // directions staged in LDS
    constexpr int SCAL = ndirs<LD>() * NF;    // offset of the staged 1/J and source
    static_assert(!RK || NPT == 1, "a fused Runge-Kutta stage needs one node per thread");
    T* __restrict__ sD = smem;
    T* __restrict__ sF = smem + Shape<NQ>::template d_slots<T>();
    const int tid = threadIdx.x;

    for (int x = tid; x < NQ2; x += NT)
        sD[x] = B.D[x];
    if constexpr (RREG)
        __syncthreads();   // phase 1 applies D along r

    RkNode<T, RK> rn;
    // phase 1 for tile node t: pointwise work and the active directions'
    // fluxes into LDS (the r contraction itself when it runs in registers,
    // into accr); returns 1/J and the source
    auto phase1 = [&](int t, T& jinv, T& src, T (&accr)[NF]) {
        const int es = t / M;
        const int m = t - es * M;
        NodeState<T, NF> st;
        load_node<T, M, NF, DIRS, GEOE>(B, ph, e0 + es, m, st);
        rn.load(B, rk, e0 + es, m, M, st);
        T* __restrict__ F = sF + es * (VPN * M) + m;
        if constexpr (RREG) {
            T fr[NF];
            put_flux<T, 1, NF>(st, 0, fr);
            contract_r_lanes<T, NQ, NF>(sD, fr, m % NQ, accr);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if ((LD >> d) & 1)
                put_flux<T, M, NF>(st, d, F + dir_slot<LD>(d) * (NF * M));
        jinv = st.jinv;
        src = st.src;
    };
    // phase 2 for tile node t: D along the active directions out of LDS
    auto phase2 = [&](int t, T jinv, T src, const T (&accr)[NF]) {
        const int es = t / M;
        const int m = t - es * M;
        const int i = m % NQ;
        const int j = (m / NQ) % NQ;
        const int k = m / NQ2;
        const T* __restrict__ Fe = sF + es * (VPN * M);
        T acc[NF];
#pragma unroll
        for (int b = 0; b < NF; ++b)
            acc[b] = accr[b];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if ((LD >> d) & 1)
                contract_dir<T, NQ, M, NF, UNR>(sD, Fe + dir_slot<LD>(d) * (NF * M), d, i, j, k,
                                                acc);
        store_node<T, M, NF, ACC, RK>(B, rk, e0 + es, m, acc, jinv, src, rn);
    };

    if constexpr (NPT == 1) {
        const bool live = tid < NODES && tid / M < ne;
        T jinv = (T)0, src = (T)0;
        T accr[NF];
#pragma unroll
        for (int b = 0; b < NF; ++b)
            accr[b] = (T)0;
        if (live)
            phase1(tid, jinv, src, accr);
        __syncthreads();
        if (live)
            phase2(tid, jinv, src, accr);
    } else {
#pragma unroll 1
        for (int t = tid; t < NODES; t += NT) {
            if (t / M < ne) {
                T jinv, src;
                T accr[NF];   // stays zero: several nodes per thread keep r in LDS
#pragma unroll
                for (int b = 0; b < NF; ++b)
                    accr[b] = (T)0;
                phase1(t, jinv, src, accr);
                const int es = t / M;
                T* S = sF + es * (VPN * M) + SCAL * M + (t - es * M);
                S[0] = jinv;
                S[M] = src;
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int t = tid; t < NODES; t += NT) {
            if (t / M < ne) {
                const int es = t / M;
                const T* S = sF + es * (VPN * M) + SCAL * M + (t - es * M);
                const T zero[NF] = {};
                phase2(t, S[0], S[M], zero);
            }
        }
    }
}

// SURF: rhs = v + s, with the neighbour faces staged in sv.sFace during the
// state loads and the face terms added in the epilogue (five fields, all
// three directions).
template <typename T, int NQ, int EPB, int NT, bool ACC, bool RK, int NF, int DIRS, bool GEOE,
          int UNR = 2, bool SURF = false>
__device__ __forceinline__ void volume_tile_alias(const BlockPtrs<T>& B, int64_t e0, int ne,
                                                  const Phys& ph, const RkStage& rk,
                                                  T* __restrict__ smem,
                                                  const SurfIn<T>& sv = SurfIn<T>{})
{
    static_assert(!SURF || (NF == 5 && DIRS == 7 && !GEOE), "the fused surface term is for the "
                                                            "five-field r+s+t volume term");
    constexpr int NQ2 = Shape<NQ>::NQ2;
    constexpr int M = Shape<NQ>::M;
    constexpr int NODES = EPB * M;
    constexpr int NPT = nodes_per_thread<NQ, EPB, NT>();
    static_assert(NPT <= alias_max_nodes_per_thread<T>(),
                  "ALIAS tiles keep every node's state of a thread in registers");
    T* __restrict__ sD = smem;
    T* __restrict__ sF = smem + Shape<NQ>::template d_slots<T>();
    const int tid = threadIdx.x;

    constexpr bool RREG = r_in_registers<NQ, EPB, NT, ALIAS, DIRS>();
    constexpr int LD = lds_dirs<NQ, EPB, NT, ALIAS, DIRS>();   // directions staged in LDS
    for (int x = tid; x < NQ2; x += NT)
        sD[x] = B.D[x];
    if constexpr (RREG)
        __syncthreads();   // D along r is applied before any LDS pass

    NodeState<T, NF> st[NPT];
    RkNode<T, RK> rn[NPT];
    T acc[NPT][NF];
    bool live[NPT];
#pragma unroll
    for (int p = 0; p < NPT; ++p) {
        const int t = tid + p * NT;
        live[p] = t < NODES && t / M < ne;
#pragma unroll
        for (int b = 0; b < NF; ++b)
            acc[p][b] = (T)0;
        if (live[p]) {
            const int es = t / M;
            load_node<T, M, NF, DIRS, GEOE, true, true, SURF>(B, ph, e0 + es, t - es * M, st[p]);
            rn[p].load(B, rk, e0 + es, t - es * M, M, st[p]);
        }
    }
    if constexpr (SURF) {
        stage_neighbour_faces<T, NQ, EPB, NT>(B, sv.nbr, ph, e0, ne, sv.sFace);
#pragma unroll
        for (int p = 0; p < NPT; ++p)
            if (live[p]) {
                const int t = tid + p * NT;
                const int es = t / M;
                const int m = t - es * M;
                stage_own_faces<T, NQ>(st[p], m % NQ, (m / NQ) % NQ, m / NQ2, (T)ph.gamma,
                                       sv.sOwn + es * (kOwnVals * 6 * NQ2));
            }
    }
    if constexpr (RREG) {
#pragma unroll
        for (int p = 0; p < NPT; ++p)
            if (live[p]) {
                const int t = tid + p * NT;
                T fr[NF];
                put_flux<T, 1, NF>(st[p], 0, fr);
                contract_r_lanes<T, NQ, NF>(sD, fr, (t - (t / M) * M) % NQ, acc[p]);
            }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (!((LD >> d) & 1))
            continue;
        if (dir_slot<LD>(d) > 0)
            __syncthreads();   // every read of the previous direction is done
#pragma unroll
        for (int p = 0; p < NPT; ++p)
            if (live[p]) {
                const int t = tid + p * NT;
                const int es = t / M;
                put_flux<T, M, NF>(st[p], d, sF + es * (NF * M) + (t - es * M));
            }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < NPT; ++p)
            if (live[p]) {
                const int t = tid + p * NT;
                const int es = t / M;
                const int m = t - es * M;
                contract_dir<T, NQ, M, NF, UNR>(sD, sF + es * (NF * M), d, m % NQ, (m / NQ) % NQ,
                                                m / NQ2, acc[p]);
            }
    }
    if constexpr (SURF) {
        // the staged faces were written before the first direction's barrier
        face_fluxes<T, NQ, EPB, NT>(sv.nbr, B.Ne, e0, ne, sv.sFace, sv.sOwn);
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < NPT; ++p)
        if (live[p]) {
            const int t = tid + p * NT;
            const int es = t / M;
            if constexpr (SURF) {
                const int m = t - es * M;
                gather_face_terms<T, NQ>(m % NQ, (m / NQ) % NQ, m / NQ2,
                                         sv.sFace + es * (kFaceVals * 6 * NQ2), sv.lift, acc[p]);
            }
            store_node<T, M, NF, ACC, RK>(B, rk, e0 + es, t - es * M, acc[p], st[p].jinv,
                                          st[p].src, rn[p]);
        }
}

template <typename T, int NQ, int EPB, int NT, int LAY, bool ACC, bool RK, int NF = 5, int DIRS = 7,
          bool GEOE = false, int UNR = 2>
__device__ __forceinline__ void volume_tile(const BlockPtrs<T>& B, int64_t e0, int ne,
                                            const Phys& ph, const RkStage& rk, T* __restrict__ smem)
{
    if constexpr (LAY == ALIAS)
        volume_tile_alias<T, NQ, EPB, NT, ACC, RK, NF, DIRS, GEOE, UNR>(B, e0, ne, ph, rk, smem);
    else
        volume_tile_full<T, NQ, EPB, NT, ACC, RK, NF, DIRS, GEOE, UNR>(B, e0, ne, ph, rk, smem);
}

// ---------------------------------------------------------------------------
// r+s tile over a group of k-slices of one element: lanes over the (i, j, k)
// nodes of S consecutive slices.  The r and s contractions of slice k need
// only slice k's fluxes, so every slice group is an independent tile: the
// LDS holds 2 NF S Nq^2 values instead of the whole element's (large
// elements, Nq = 12 and 16, stay resident several workgroups per CU, FP64 at
// Nq = 16 fits), and an element spreads over Nq / S workgroups, which keeps
// the chip busy on the few large elements of a fixed node count.
// ---------------------------------------------------------------------------
// Slices per workgroup and unroll of the contraction loop, per precision and
// Nq, as measured on MI355X (8 fields, r+s, the fixed-node-count shapes):
// FP32 at Nq = 12 takes two slices (288 of 320 lanes live), every other
// shape one slice.  Fewer contraction terms are kept in flight where the
// whole loop would not fit the register budget (FP64 at Nq = 16, four waves
// per SIMD; FP32 with 5 fields at Nq = 16, eight waves).
template <typename T, int NQ>
constexpr int slab_slices()
{
    return (sizeof(T) == 4 && NQ == 12) ? 2 : 1;
}

template <typename T, int NQ, int NF>
constexpr int slab_unroll()
{
    if constexpr (sizeof(T) == 4)
        return NQ == 12 ? 2 : (NF == 8 ? NQ : 8);
    else
        return NQ == 16 ? 8 : NQ;
}

template <typename T, int NQ>
constexpr int slab_threads()
{
    return ((slab_slices<T, NQ>() * NQ * NQ + 63) / 64) * 64;
}

template <typename T, int NQ, int NF>
constexpr int volume_slab_lds_values()
{
    return Shape<NQ>::template d_slots<T>() + 2 * NF * slab_slices<T, NQ>() * NQ * NQ;
}

// Slice groups g = 0 .. Ne Nq / S - 1, group g covering slices
// k0 .. k0 + S - 1 of element g / (Nq / S), k0 = S (g mod Nq / S); the
// workgroups stride over them.
template <typename T, int NQ, bool ACC, int NF, bool GEOE>
__device__ __forceinline__ void volume_tile_slab(const BlockPtrs<T>& B, const Phys& ph,
                                                 T* __restrict__ smem)
{
    constexpr int NQ2 = Shape<NQ>::NQ2;
    constexpr int M = Shape<NQ>::M;
    constexpr int S = slab_slices<T, NQ>();
    constexpr int G = NQ / S;   // slice groups per element
    constexpr int NT = slab_threads<T, NQ>();
    constexpr int UNR = slab_unroll<T, NQ, NF>();
    // the group's run of each array is whole 128-byte lines (streamed), or
    // shares lines with the next group's (read through the cache)
    constexpr bool STREAM = (S * NQ2 * (int)sizeof(T)) % 128 == 0;
    T* __restrict__ sD = smem;
    T* __restrict__ sF = smem + Shape<NQ>::template d_slots<T>();
    const int tid = threadIdx.x;
    for (int x = tid; x < NQ2; x += NT)
        sD[x] = B.D[x];
    const bool live = tid < S * NQ2;
    const int ks = tid / NQ2;              // slice within the group
    const int ij = tid - ks * NQ2;
    const int i = ij % NQ, j = ij / NQ;
    T* __restrict__ sFr = sF + ks * (2 * NF * NQ2);
    T* __restrict__ sFs = sFr + NF * NQ2;
    const RkStage no_rk{0.0, 0.0, 0.0};
    const RkNode<T, false> no_rn{};
    const int64_t groups = B.Ne * G;
#pragma unroll 1
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t e = g / G;
        const int m = tid + NQ2 * S * (int)(g - e * G);
        NodeState<T, NF> st;
        if (g != (int64_t)blockIdx.x)
            __syncthreads();   // the previous group's reads of the slice buffer are done
        if (live) {
            load_node<T, M, NF, 3, GEOE, STREAM>(B, ph, e, m, st);
            put_flux<T, NQ2, NF>(st, 0, sFr + ij);
            put_flux<T, NQ2, NF>(st, 1, sFs + ij);
        }
        __syncthreads();
        if (live) {
            T acc[NF];
#pragma unroll
            for (int b = 0; b < NF; ++b)
                acc[b] = (T)0;
            contract<T, NQ, NQ2, NF, UNR>(sD, sFr + NQ * j, i, 1, acc);
            contract<T, NQ, NQ2, NF, UNR>(sD, sFs + i, j, NQ, acc);
            store_node<T, M, NF, ACC, false, STREAM>(B, no_rk, e, m, acc, st.jinv, st.src, no_rn);
        }
    }
}

// ---------------------------------------------------------------------------
// t term of large elements as a pass of its own: rhs += -(1/J) D_t F^t, with
// no source (the r+s pass before it wrote the rest).  The t contraction
// couples only the Nq nodes of one (i, j) column, so a tile is a block of
// J rows of columns, (i, j0 .. j0 + J - 1, all k): Nq^2 J nodes, one per
// lane, their t fluxes in LDS.  For each k the block's nodes are J Nq
// consecutive values of every array.
// ---------------------------------------------------------------------------
template <typename T, int NQ>
constexpr int tcol_rows()
{
    return 2;
}

template <typename T, int NQ>
constexpr int tcol_threads()
{
    return NQ * NQ * tcol_rows<T, NQ>();
}

template <typename T, int NQ, int NF>
constexpr int volume_tcol_lds_values()
{
    return Shape<NQ>::template d_slots<T>() + NF * tcol_threads<T, NQ>();
}

template <typename T, int NQ, int NF, bool GEOE>
__device__ __forceinline__ void volume_tile_tcol(const BlockPtrs<T>& B, const Phys& ph,
                                                 T* __restrict__ smem)
{
    constexpr int NQ2 = Shape<NQ>::NQ2;
    constexpr int M = Shape<NQ>::M;
    constexpr int J = tcol_rows<T, NQ>();
    constexpr int G = NQ / J;            // column blocks per element
    constexpr int NT = tcol_threads<T, NQ>();
    constexpr int ROW = J * NQ;          // nodes of one k in the block
    constexpr bool STREAM = (ROW * (int)sizeof(T)) % 128 == 0;
    static_assert(NQ % J == 0, "column blocks tile the element");
    T* __restrict__ sD = smem;
    T* __restrict__ sF = smem + Shape<NQ>::template d_slots<T>();
    const int tid = threadIdx.x;
    for (int x = tid; x < NQ2; x += NT)
        sD[x] = B.D[x];
    const int k = tid / ROW;
    const int c = tid - k * ROW;         // column within the block: i + Nq jj
    const RkStage no_rk{0.0, 0.0, 0.0};
    const RkNode<T, false> no_rn{};
    const int64_t groups = B.Ne * G;
#pragma unroll 1
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t e = g / G;
        const int m = NQ * J * (int)(g - e * G) + c + NQ2 * k;
        NodeState<T, NF> st;
        if (g != (int64_t)blockIdx.x)
            __syncthreads();   // the previous block's reads of the flux buffer are done
        load_node<T, M, NF, 4, GEOE, STREAM, false>(B, ph, e, m, st);
        put_flux<T, NT, NF>(st, 2, sF + tid);
        __syncthreads();
        T acc[NF];
#pragma unroll
        for (int b = 0; b < NF; ++b)
            acc[b] = (T)0;
        contract<T, NQ, NT, NF, (sizeof(T) == 4 ? NQ : 8)>(sD, sF + c, k, ROW, acc);
        store_node<T, M, NF, true, false, STREAM>(B, no_rk, e, m, acc, st.jinv, (T)0, no_rn);
    }
}

// ---------------------------------------------------------------------------
// Column-sweep tile: one element per Nq^2 lanes, lane (i, j) owning the
// column of nodes (i, j, 0 .. Nq-1), walking the element slice by slice
// (k = n) with the next slice's loads in flight.  Slice n's r and s
// contractions complete its outputs' r+s sums at once; its t fluxes
// contribute D[k][n] F^t(i, j, n) to every output k of the lane's column,
// kept in registers, so the t contraction needs no LDS and every input is
// read once and every output written once, with LDS holding only one slice
// of r and s fluxes (double-buffered) and the 1/J and source of the column.
// r and s run out of LDS (a lane's r line is read by the whole row of
// lanes, one broadcast per value; DPP row rotations instead measured no
// faster, their moves and hazard waits taking VALU issue slots).
// ---------------------------------------------------------------------------
template <int NQ>
constexpr bool sweep_supported()
{
    return NQ == 8 || NQ == 16;
}

// elements per workgroup: four waves
template <int NQ>
constexpr int sweep_elems()
{
    return NQ * NQ >= 256 ? 1 : 256 / (NQ * NQ);
}

template <typename T, int NQ, int NF>
constexpr int sweep_lds_values()
{
    constexpr int NQ2 = NQ * NQ;
    // D, D transposed, two slices of s and r fluxes, 1/J and source per node
    return 2 * Shape<NQ>::template d_slots<T>() + sweep_elems<NQ>() * (4 * NF * NQ2 + 2 * NQ * NQ2);
}

// Loads of one node, kept raw so that the next slice's can be in flight.
template <typename T, int NF, bool GEOE>
struct SweepRaw {
    T q[NF];
    T g[GEOE ? 1 : 10];
    T rr;
    double thr;
};

template <typename T, int NQ, int NF, bool ACC, bool GEOE>
__device__ __forceinline__ void volume_tile_sweep(const BlockPtrs<T>& B, const Phys& ph,
                                                  T* __restrict__ smem)
{
    static_assert(sweep_supported<NQ>(), "elements of 8 or 16 nodes per line");
    constexpr int NQ2 = NQ * NQ;
    constexpr int M = NQ2 * NQ;
    constexpr int EPW = sweep_elems<NQ>();
    constexpr int NT = EPW * NQ2;
    constexpr int DS = Shape<NQ>::template d_slots<T>();
    T* __restrict__ sD = smem;              // D[i][n]
    T* __restrict__ sDT = smem + DS;        // D[k][n] at n * NQ + k
    // s fluxes [2][EPW][NF][NQ2], then r fluxes of the same shape
    T* __restrict__ sFs = smem + 2 * DS;
    T* __restrict__ sJS = sFs + 4 * EPW * NF * NQ2;   // [EPW][NQ][2][NQ2]
    const int tid = threadIdx.x;
    for (int x = tid; x < NQ2; x += NT) {
        const T v = B.D[x];
        sD[x] = v;
        sDT[(x % NQ) * NQ + x / NQ] = v;
    }
    const int es = tid / NQ2;
    const int l = tid - es * NQ2;
    const int i = l % NQ, j = l / NQ;
    const int64_t e = (int64_t)blockIdx.x * EPW + es;
    const bool live = e < B.Ne;
    const bool has_ref = B.theta_ref != nullptr;
    // per-element metric record (affine elements): one per wave
    T ge[10];
    if constexpr (GEOE) {
        const int64_t eu = __builtin_amdgcn_readfirstlane((int)(live ? e : 0));
#pragma unroll
        for (int s = 0; s < 10; ++s)
            ge[s] = B.geo[eu * 10 + s];
    }
    auto load = [&](int n, SweepRaw<T, NF, GEOE>& r) {
        const int m = l + NQ2 * n;
        const T* __restrict__ qe = B.q + e * (NF * M) + m;
#pragma unroll
        for (int b = 0; b < NF; ++b)
            r.q[b] = ld_stream(qe + b * M);
        if constexpr (!GEOE) {
            const T* __restrict__ gp = B.geo + e * (10 * M) + m;
#pragma unroll
            for (int s = 0; s < 10; ++s)
                r.g[s] = ld_stream(gp + s * M);
        }
        r.rr = (T)0;
        r.thr = 0.0;
        if (has_ref) {
            r.rr = ld_stream(B.rho_ref + e * M + m);
            r.thr = ld_stream(B.theta_ref + e * M + m);
        }
    };
    T acc[NQ][NF];
#pragma unroll
    for (int k = 0; k < NQ; ++k)
#pragma unroll
        for (int b = 0; b < NF; ++b)
            acc[k][b] = (T)0;
    SweepRaw<T, NF, GEOE> cur, nxt;
    if (live)
        load(0, cur);
    __syncthreads();   // D and D^T staged
    T* __restrict__ JS = sJS + es * (2 * NQ * NQ2) + l;
    // unrolled by two: the prefetched slice alternates between two register
    // sets instead of being copied (Nq = 16, 8 fields: 133 -> 119 us)
#pragma unroll 2
    for (int n = 0; n < NQ; ++n) {
        if (live && n + 1 < NQ)
            load(n + 1, nxt);
        T* __restrict__ Fs = sFs + ((n & 1) * EPW + es) * (NF * NQ2);
        T* __restrict__ Fr = sFs + ((2 + (n & 1)) * EPW + es) * (NF * NQ2);
        T rs[NF];
#pragma unroll
        for (int b = 0; b < NF; ++b)
            rs[b] = (T)0;
        if (live) {
            NodeState<T, NF> st;
            st.rho = cur.q[0];
            st.U1 = cur.q[1];
            st.U2 = cur.q[2];
            st.U3 = cur.q[3];
            st.Th = cur.q[4];
#pragma unroll
            for (int b = 5; b < NF; ++b)
                st.Q[b - 5] = cur.q[b];
#pragma unroll
            for (int s = 0; s < 9; ++s)
                st.g[s] = GEOE ? ge[s] : cur.g[s];
            st.jinv = GEOE ? ge[9] : cur.g[9];
            st.src = -(T)ph.grav * (st.rho - cur.rr);
            st.pp = Pressure<T>::eval(st.Th, has_ref, cur.thr, ph);
            st.rinv = recip(st.rho);
            JS[n * (2 * NQ2)] = st.jinv;
            JS[n * (2 * NQ2) + NQ2] = st.src;
            T f[NF];
            put_flux<T, NQ2, NF>(st, 1, Fs + l);       // s fluxes to LDS
            put_flux<T, NQ2, NF>(st, 0, Fr + l);       // r fluxes to LDS
            put_flux<T, 1, NF>(st, 2, f);              // t fluxes: to every output k
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const T dkn = sDT[n * NQ + k];
#pragma unroll
                for (int b = 0; b < NF; ++b)
                    acc[k][b] += dkn * f[b];
            }
        }
        __syncthreads();   // slice n's s (and r) fluxes are visible
        if (live) {
            contract<T, NQ, NQ2, NF, NQ>(sD, Fr + NQ * j, i, 1, rs);
#pragma unroll
            for (int m2 = 0; m2 < NQ; ++m2) {
                const T dm = sD[j * NQ + m2];
#pragma unroll
                for (int b = 0; b < NF; ++b)
                    rs[b] += dm * Fs[b * NQ2 + i + NQ * m2];
            }
            // the r+s sums belong to output k = n
#pragma unroll
            for (int k = 0; k < NQ; ++k)
                if (k == n) {
#pragma unroll
                    for (int b = 0; b < NF; ++b)
                        acc[k][b] += rs[b];
                }
        }
        cur = nxt;
    }
    if (!live)
        return;
    const int64_t base = e * (NF * M) + l;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const T jinv = JS[k * (2 * NQ2)];
        const T src = JS[k * (2 * NQ2) + NQ2];
        T* __restrict__ re = B.rhs + base + k * NQ2;
#pragma unroll
        for (int b = 0; b < NF; ++b) {
            T v = -jinv * acc[k][b];
            if (b == 3)
                v += src;
            if constexpr (ACC)
                v += ld_stream(re + b * M);
            st_stream(re + b * M, v);
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint tile (vector-Jacobian product with respect to q).
//   w_b(x)   = -(1/J(x)) lambda_b(x)                       (phase 1, to LDS)
//   G^d_b(y) = sum_x Dd[x][y] w_b(x)   along r, s, t       (phase 2, D^T)
//   with v^d = U^d/rho and A^d = sum_a G^d_{Ua} U_a + G^d_Theta Theta:
//   mu_rho = -(1/rho) sum_d v^d A^d - grav lambda_U3
//   mu_Uc  = sum_d [ g_cd (G^d_rho + A^d/rho) + v^d G^d_Uc ]
//   mu_Th  = sum_d [ (dp/dTheta) sum_a g_ad G^d_Ua + v^d G^d_Theta ]
// ---------------------------------------------------------------------------
template <typename T>
struct AdjPtrs {
    const T* D;
    const T* geo;
    const T* q;
    const T* lambda;
    T* mu;
    int64_t Ne;
};

// Pointwise inputs of one adjoint node, read in phase 1 together with lambda
// so that every global load of the tile is in flight before the barrier.
template <typename T>
struct AdjNode {
    T U1, U2, U3, Th, rinv, dpdT, lam3;
    T g[9];
};

template <typename T, int NQ, int EPB, int NT, bool ACC>
__device__ __forceinline__ void adjoint_tile(const AdjPtrs<T>& B, int64_t e0, int ne,
                                             const Phys& ph, T* __restrict__ smem)
{
    constexpr int NQ2 = Shape<NQ>::NQ2;
    constexpr int M = Shape<NQ>::M;
    constexpr int NODES = EPB * M;
    constexpr int NPT = (NODES + NT - 1) / NT;
    T* __restrict__ sD = smem;
    T* __restrict__ sW = smem + Shape<NQ>::template d_slots<T>();
    const int tid = threadIdx.x;

    for (int x = tid; x < NQ2; x += NT)
        sD[x] = B.D[x];

    AdjNode<T> nd[NPT];
#pragma unroll
    for (int p = 0; p < NPT; ++p) {
        const int t = tid + p * NT;
        const int es = t / M;
        const int m = t - es * M;
        if (t < NODES && es < ne) {
            const int64_t e = e0 + es;
            const T* __restrict__ le = B.lambda + e * (5 * M) + m;
            const T* __restrict__ qe = B.q + e * (5 * M) + m;
            const T* __restrict__ ge = B.geo + e * (10 * M) + m;
            T lb[5];
#pragma unroll
            for (int b = 0; b < 5; ++b)
                lb[b] = ld_stream(le + b * M);
            const T jinv = ld_stream(ge + 9 * M);
            const T rho = ld_stream(qe);
            nd[p].U1 = ld_stream(qe + M);
            nd[p].U2 = ld_stream(qe + 2 * M);
            nd[p].U3 = ld_stream(qe + 3 * M);
            nd[p].Th = ld_stream(qe + 4 * M);
#pragma unroll
            for (int s = 0; s < 9; ++s)
                nd[p].g[s] = ld_stream(ge + s * M);
            T* W = sW + es * (5 * M) + m;
#pragma unroll
            for (int b = 0; b < 5; ++b)
                W[b * M] = -jinv * lb[b];
            nd[p].lam3 = lb[3];
            nd[p].rinv = recip(rho);
            nd[p].dpdT = Pressure<T>::dp_dtheta(nd[p].Th, ph);
        }
    }
    __syncthreads();

#pragma unroll
    for (int p = 0; p < NPT; ++p) {
        const int t = tid + p * NT;
        const int es = t / M;
        const int m = t - es * M;
        if (t < NODES && es < ne) {
            const int i = m % NQ;
            const int j = (m / NQ) % NQ;
            const int k = m / NQ2;
            const int64_t e = e0 + es;
            const AdjNode<T>& n = nd[p];
            const T* __restrict__ We = sW + es * (5 * M);
            T G[3][5];
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int b = 0; b < 5; ++b)
                    G[d][b] = (T)0;
            {   // r: G^r(i,j,k) = sum_x D[x][i] w(x, j, k)
                const T* Wr = We + NQ * j + NQ2 * k;
#pragma unroll 2
                for (int x = 0; x < NQ; ++x) {
                    const T dx = sD[x * NQ + i];
#pragma unroll
                    for (int b = 0; b < 5; ++b)
                        G[0][b] += dx * Wr[b * M + x];
                }
            }
            {   // s: G^s(i,j,k) = sum_x D[x][j] w(i, x, k)
                const T* Ws = We + i + NQ2 * k;
#pragma unroll 2
                for (int x = 0; x < NQ; ++x) {
                    const T dx = sD[x * NQ + j];
#pragma unroll
                    for (int b = 0; b < 5; ++b)
                        G[1][b] += dx * Ws[b * M + NQ * x];
                }
            }
            {   // t: G^t(i,j,k) = sum_x D[x][k] w(i, j, x)
                const T* Wt = We + i + NQ * j;
#pragma unroll 2
                for (int x = 0; x < NQ; ++x) {
                    const T dx = sD[x * NQ + k];
#pragma unroll
                    for (int b = 0; b < 5; ++b)
                        G[2][b] += dx * Wt[b * M + NQ2 * x];
                }
            }
            T mu0 = (T)0, mu1 = (T)0, mu2 = (T)0, mu3 = (T)0, mu4 = (T)0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const T g1 = n.g[3 * d], g2 = n.g[3 * d + 1], g3 = n.g[3 * d + 2];
                const T vd = (g1 * n.U1 + g2 * n.U2 + g3 * n.U3) * n.rinv;
                const T Ad = G[d][1] * n.U1 + G[d][2] * n.U2 + G[d][3] * n.U3 + G[d][4] * n.Th;
                const T cd = G[d][0] + Ad * n.rinv;
                mu0 += vd * Ad;
                mu1 += g1 * cd + vd * G[d][1];
                mu2 += g2 * cd + vd * G[d][2];
                mu3 += g3 * cd + vd * G[d][3];
                mu4 += n.dpdT * (g1 * G[d][1] + g2 * G[d][2] + g3 * G[d][3]) + vd * G[d][4];
            }
            mu0 = -n.rinv * mu0 - (T)ph.grav * n.lam3;
            T* __restrict__ me = B.mu + e * (5 * M) + m;
            const T out[5] = {mu0, mu1, mu2, mu3, mu4};
#pragma unroll
            for (int b = 0; b < 5; ++b) {
                T v = out[b];
                if constexpr (ACC)
                    v += ld_stream(me + b * M);
                st_stream(me + b * M, v);
            }
        }
    }
}

}  // namespace semk
