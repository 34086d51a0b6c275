/*
 * semvol — the strong-form spectral-element volume term of the dry-atmosphere
 * Euler equations on one AMD Instinct MI355X (gfx950).
 *
 * The operation is the one of Sec. 2 of Klöckner, Wilcox, Warburton, "Array
 * Program Transformation with Loo.py by Example: High-Order Finite Elements"
 * (ARRAY'16): the volume contribution v of Eq. (volterm) to the method-of-lines
 * rate dq/dt = v(q) + s(q), for hexahedral elements of Nq^3 Gauss-Lobatto
 * nodes, with the flux column of equation set 2C and the equation of state
 * p = p0 (R Theta / p0)^gamma (Sec. 2).  This library adds a gravity source,
 * a reference-state (perturbation) pressure, an FP32 form, a vector-Jacobian
 * product, a mixed-order batched launch and an SSP-RK3 step captured in a
 * HIP graph.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *   Nq            nodes per direction (polynomial order N = Nq - 1); supported
 *                 2 <= Nq <= 10.
 *   node index    m = i + Nq*j + Nq^2*k, with i, j, k along the reference
 *                 directions r, s, t (Fig. 1 of the paper).
 *   D             [Nq][Nq], D[i*Nq + n] = l_n'(xi_i): row i is the output node.
 *   geo           [Ne][10][Nq^3]: slot 3*d + a holds g_{a d} = J * dxi_d/dx_a
 *                 (a, d = 0..2; slots 0-2 serve the r sum, 3-5 the s sum, 6-8
 *                 the t sum, as in the listed r/s kernels), slot 9 holds 1/J.
 *   q, rhs        [Ne][5][Nq^3]: rho, U1 = rho u, U2 = rho v, U3 = rho w,
 *                 Theta = rho theta (the order of the prognostic vector).
 *   rho_ref       [Ne][Nq^3], same dtype as q, or NULL.
 *   theta_ref     [Ne][Nq^3], ALWAYS FP64, or NULL.  rho_ref and theta_ref are
 *                 both NULL or both given.
 *   dtype         SEM_F64: every array FP64.  SEM_F32: D, geo, q, rho_ref,
 *                 rhs, lambda, mu FP32; theta_ref stays FP64.
 *
 * The computed volume term (readings of Sec. 2 where it is silent):
 *   v_b(i,j,k) = -(1/J(i,j,k)) sum_{n,a} [ D[i][n] g_a0(n,j,k) f_ab(n,j,k)
 *                                        + D[j][n] g_a1(i,n,k) f_ab(i,n,k)
 *                                        + D[k][n] g_a2(i,j,n) f_ab(i,j,n) ]
 *   v_U3      += -grav * (rho - rho_ref)
 * with f_a the flux column of set 2C (5 fields) and the pressure in f replaced
 * by p - p_ref, p_ref = p0 (R Theta_ref / p0)^gamma, when a reference is given
 * (rho_ref = 0 and p_ref = 0 otherwise).  The sign is the one of the listed
 * kernels and of dq/dt = -div f (Eq. (volterm) prints "+").
 *
 * Memory and streams: every array argument is a DEVICE pointer owned by the
 * caller and must stay valid until the enqueued work has finished.  Pointers
 * must be aligned to their element size.  `stream` is a hipStream_t (NULL =
 * the null stream).  Calls only enqueue work; none synchronises except
 * sem_batch_plan and sem_rk3_graph_create when they autotune.
 *
 * Errors: every entry point returns a sem_status.  Arguments are validated on
 * the host before any HIP call; on failure nothing is enqueued and
 * sem_last_error() returns a message.  A failed kernel launch returns
 * SEM_ERR_HIP.  Numerical domain errors (rho = 0, Theta <= 0) are not
 * checked: NaN/Inf propagate to the outputs of the affected element.
 */
#ifndef SEMVOL_SEM_H
#define SEMVOL_SEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sem_status {
    SEM_OK = 0,
    SEM_ERR_INVALID_ARG = -1,   /* bad size, NULL or misaligned pointer, bad dtype */
    SEM_ERR_UNSUPPORTED = -2,   /* Nq or tile shape not compiled in */
    SEM_ERR_HIP = -3,           /* a HIP runtime call or kernel launch failed */
    SEM_ERR_NO_MEMORY = -4      /* host or device allocation failed (plans, graphs) */
} sem_status;

/* Element type of the arrays.  An int32_t rather than an enum, so that any
 * value a caller passes is well defined inside the library and rejected with
 * SEM_ERR_INVALID_ARG unless it is one of these. */
typedef int32_t sem_dtype;
#define SEM_F64 0
#define SEM_F32 1

/* Physical constants: the paper's kernel arguments p_p0, p_Gamma, p_R
 * (reference pressure, ratio of specific heats, gas constant), plus the
 * gravitational acceleration of the source term. */
typedef struct sem_phys {
    double p0;
    double gamma;
    double R;
    double grav;
} sem_phys;

/* Tile shape of the single-order kernels: elements per workgroup and LDS
 * layout.  SEM_LAYOUT_FULL stages the contravariant fluxes of all three
 * reference directions in LDS (one barrier); SEM_LAYOUT_ALIAS stages one
 * direction at a time (a third of the LDS, three barriers).  Zeros select the
 * built-in default for (dtype, Nq), the fastest compiled shape measured on
 * MI355X; a zero element count with an explicit layout takes the default's
 * count when that shape exists (else the smallest compiled one), and an
 * explicit count with SEM_LAYOUT_DEFAULT takes FULL if compiled, else ALIAS. */
#define SEM_LAYOUT_DEFAULT 0
#define SEM_LAYOUT_FULL 1
#define SEM_LAYOUT_ALIAS 2
typedef struct sem_tile {
    int32_t elems_per_block;
    int32_t layout;
} sem_tile;

/* Thread-local text describing the last non-OK status of this thread. */
const char* sem_last_error(void);

/* Library version string. */
const char* sem_version(void);

/*
 * Volume term of Eq. (volterm) plus the gravity source, for Ne elements of
 * one order (the argument list of the paper's refFluxR/refFluxS kernels,
 * (Ne, Nq, geo, D, q, rhsq, p_p0, p_Gamma, p_R), extended by dtype, the
 * reference state, gravity and a stream).
 *   rhs = v(q)            if accumulate == 0
 *   rhs = rhs + v(q)      otherwise (the paper's rhsq update semantics)
 * No byte of rhs may lie inside q, geo, D or the reference arrays (their
 * extents follow from Ne, Nq and dtype).
 * Errors: Ne < 1 (the paper's assumption Ne >= 1), unsupported Nq, NULL
 * required pointer, only one of rho_ref/theta_ref, misaligned pointer, rhs
 * overlapping an input, unknown dtype -> SEM_ERR_INVALID_ARG /
 * SEM_ERR_UNSUPPORTED before any HIP call.  Allocates nothing and enqueues only kernel launches (no memset or
 * copy), so a caller may capture it into a HIP graph.
 */
sem_status sem_volume_rhs(int32_t Ne, int32_t Nq, sem_dtype dtype,
                          const void* D, const void* geo, const void* q,
                          const void* rho_ref, const double* theta_ref,
                          const sem_phys* phys, void* rhs, int32_t accumulate,
                          void* stream);

/* As sem_volume_rhs, with an explicit tile shape (NULL = default).  A shape
 * that is not compiled for (dtype, Nq) returns SEM_ERR_UNSUPPORTED, an
 * unknown layout code SEM_ERR_INVALID_ARG.  Every shape computes the same
 * values (up to the order of floating-point additions). */
sem_status sem_volume_rhs_tiled(int32_t Ne, int32_t Nq, sem_dtype dtype,
                                const void* D, const void* geo, const void* q,
                                const void* rho_ref, const double* theta_ref,
                                const sem_phys* phys, void* rhs, int32_t accumulate,
                                const sem_tile* tile, void* stream);

/* Caps the number of workgroups of the strided launches (the k-slice and
 * t-column passes of sem_volume_rhs_ext and sem_volume_rhs_affine at
 * Nq >= 12) for the whole process; 0 (the default) leaves one workgroup per
 * tile.  A cap leaves compute units free for concurrent work and lets tests
 * exercise the strided path at small sizes; results do not depend on it.
 * Errors: cap < 0 -> SEM_ERR_INVALID_ARG. */
sem_status sem_set_max_workgroups(int64_t cap);

/* Writes up to `cap` compiled tile shapes for (dtype, Nq) into `out` and
 * returns how many exist (0 for an unsupported Nq or dtype). */
int32_t sem_tile_options(sem_dtype dtype, int32_t Nq, sem_tile* out, int32_t cap);

/*
 * Extended volume term: the full prognostic vector of Sec. 2 with the three
 * passive tracers Q1..Q3 (flux U_a Q_i / rho), and the choice of the reference
 * directions that enter Eq. (volterm).  The paper's benchmark kernel fuses
 * the r and s terms of 8 fields (nfields = 8, dirs = SEM_DIR_R | SEM_DIR_S).
 *   nfields   5 (rho, U1, U2, U3, Theta) or 8 (plus Q1, Q2, Q3);
 *             q, rhs: [Ne][nfields][Nq^3]
 *   dirs      SEM_DIR_R | SEM_DIR_S, or SEM_DIR_R | SEM_DIR_S | SEM_DIR_T; the
 *             geo slots of an excluded direction are not read
 *   Nq        2..10, 12 or 16
 * All other arguments, the gravity source and the reference state are as for
 * sem_volume_rhs.  Each (Nq, nfields, dirs) has one built-in tile shape; r+s at
 * Nq >= 12 tiles each element by groups of k-slices.  r+s+t at Nq = 16 is two
 * launches on `stream`: the r+s term with the source (as requested, overwrite
 * or accumulate), then the t term added to it; the result is the same up to
 * rounding order (the t sum is added to the finished r+s value instead of
 * being summed with it before the 1/J factor).  These passes launch one
 * workgroup per tile up to a cap (2^32 work-items, or the cap set with
 * sem_set_max_workgroups if lower); the workgroups then stride over the
 * tiles.
 * Errors: unsupported nfields / dirs / Nq -> SEM_ERR_UNSUPPORTED; otherwise as
 * sem_volume_rhs.  Allocates nothing.
 */
#define SEM_DIR_R 1u
#define SEM_DIR_S 2u
#define SEM_DIR_T 4u
sem_status sem_volume_rhs_ext(int32_t Ne, int32_t Nq, sem_dtype dtype, int32_t nfields,
                              uint32_t dirs, const void* D, const void* geo, const void* q,
                              const void* rho_ref, const double* theta_ref,
                              const sem_phys* phys, void* rhs, int32_t accumulate,
                              void* stream);

/*
 * Optimisation ladder (the analogue of the per-level timings of Sec. 4,
 * Table 1) of the paper's benchmark kernel: the fused r+s volume term of
 * Eq. (volterm) with the 8-field prognostic vector of Sec. 2, FP32, no
 * reference state and no source, accumulated:
 *   rhs += -(1/J) sum_{d in r,s} D_d (sum_a g_ad f_a)
 * Every level computes the same values (up to FP32 rounding order):
 *   1  naive: per output node and per n, state, metric terms, pressure and
 *      flux at the line node from global memory, D from global memory, rhs
 *      read-modify-written in global memory for every term;
 *   2  + D in LDS;
 *   3  + fluxes evaluated once per node into LDS, a k-slice at a time;
 *   4  + rhs accumulated in registers, one global update per output;
 *   5  + 1/J applied once per output;
 *   6  the production kernel (sem_volume_rhs_ext with nfields = 8, r+s).
 * Levels 1-5 use one workgroup per element and one lane per (i, j) node.
 *   Nq      2..10, 12, 16
 *   D, geo, q, rhs   FP32 device arrays as for sem_volume_rhs_ext (nfields 8);
 *                    geo slots 6-8 (the t direction) are not read
 *   phys    p0, gamma, R; grav must be 0
 * Errors: level outside 1..SEM_LADDER_LEVELS, Ne < 1, NULL or misaligned
 * pointers, rhs aliasing an input -> SEM_ERR_INVALID_ARG; unsupported Nq or
 * grav != 0 -> SEM_ERR_UNSUPPORTED.  Allocates nothing.
 */
#define SEM_LADDER_LEVELS 6
sem_status sem_volume_rhs_ladder(int32_t level, int32_t Ne, int32_t Nq, const void* D,
                                 const void* geo, const void* q, const sem_phys* phys,
                                 void* rhs, void* stream);

/*
 * Volume term of sem_volume_rhs for affine elements, whose metric terms g and
 * 1/J are constant in each element (Sec. 2 names them geometric factors of the
 * reference-to-physical map; for x = A xi + b they do not vary inside the
 * element):
 *   geo_elem  [Ne][10], slot 3*d + a = g_{a d}, slot 9 = 1/J, one set per element
 * Every other argument as for sem_volume_rhs; Nq 2..10, 12, 16 (Nq = 16 runs
 * as the two launches described for sem_volume_rhs_ext).  The per-node metric
 * arrays are 10 of the 22 values a node moves in FP64; this form moves 12.
 * Errors as for sem_volume_rhs.  Allocates nothing.
 */
sem_status sem_volume_rhs_affine(int32_t Ne, int32_t Nq, sem_dtype dtype, const void* D,
                                 const void* geo_elem, const void* q, const void* rho_ref,
                                 const double* theta_ref, const sem_phys* phys, void* rhs,
                                 int32_t accumulate, void* stream);

/*
 * Vector-Jacobian product of the volume term with respect to the state
 * (derivative of the flux column and EOS of Sec. 2):
 *   mu = (dv/dq)^T lambda        (mu += ... if accumulate != 0)
 * The reference state does not enter: d(p - p_ref)/dTheta = dp/dTheta.
 * lambda, mu: [Ne][5][Nq^3], dtype.  No byte of mu may lie inside D, geo,
 * q or lambda.
 * Errors as for sem_volume_rhs.  Allocates nothing.
 */
sem_status sem_volume_rhs_adjoint(int32_t Ne, int32_t Nq, sem_dtype dtype,
                                  const void* D, const void* geo, const void* q,
                                  const sem_phys* phys, const void* lambda, void* mu,
                                  int32_t accumulate, void* stream);

/*
 * Surface term s of the method-of-lines rate dq/dt = v(q) + s(q) (Sec. 2
 * splits the rate into a volume and a surface contribution and defines only
 * the volume one).  Reading taken: the strong-form discontinuous Galerkin face
 * term on the same GLL nodes, with a local Lax-Friedrichs (Rusanov) flux.  At
 * a node x of face (d, side) of element e, with N = sigma (g_0d, g_1d,
 * g_2d)(x) (sigma = -1 on the face xi_d = -1, +1 on xi_d = +1), q- the state
 * of e at x and q+ the neighbour's state at the same node:
 *   s_b(x) += -(1/J(x)) (N(N+1)/2) [ (Fn_b(q+) - Fn_b(q-)) / 2
 *                                     - lambda |N| (q+_b - q-_b) / 2 ]
 * Fn(q) = sum_a N_a f_a(q) is the flux column of set 2C with the volume term's
 * pressure (each side's p - p_ref when theta_ref is given, else p),
 * lambda = max over both sides of |u . N|/|N| + sqrt(gamma p / rho) (full p),
 * and N(N+1)/2 = 1/w_N, the inverse GLL weight of the end nodes.  Nodes on
 * edges and corners collect the terms of each of their faces.
 *   nbr        [Ne][6] int32: the element across faces r-, r+, s-, s+, t-, t+
 *              (face 2 d + side).  Meshes are conforming with aligned
 *              faces: across its r = -1 face, node (0, j, k) of e meets node
 *              (N, j, k) of nbr[e][0] (likewise for s and t).  An index
 *              outside [0, Ne) is a boundary face whose exterior state equals
 *              the interior one, so it adds nothing; the kernel never reads
 *              through such an index.
 *   geo, q     as for sem_volume_rhs (only face nodes are read)
 *   theta_ref  [Ne][Nq^3] FP64 or NULL: the reference of the pressure
 *              perturbation (where it is continuous across a face it cancels;
 *              in FP32 it keeps the pressure difference accurate)
 *   rhs        rhs = s (zero at interior nodes) if accumulate == 0, else
 *              rhs += s (after sem_volume_rhs this completes v + s)
 *   Nq         2..10, 12, 16
 * No byte of rhs may lie inside nbr, geo, q or theta_ref.
 * Errors: Ne < 1, NULL or misaligned pointer, rhs overlapping an input,
 * unknown dtype -> SEM_ERR_INVALID_ARG; unsupported Nq -> SEM_ERR_UNSUPPORTED.
 * Allocates nothing; enqueues one kernel launch.
 */
sem_status sem_surface_rhs(int32_t Ne, int32_t Nq, sem_dtype dtype, const int32_t* nbr,
                           const void* geo, const void* q, const double* theta_ref,
                           const sem_phys* phys, void* rhs, int32_t accumulate, void* stream);

/* The whole rate dq/dt = v(q) + s(q) of Sec. 2 in one kernel launch: the
 * volume term of sem_volume_rhs and the surface term of sem_surface_rhs,
 * evaluated together so that every input is read once and rhs is written
 * once.  rhs = v + s (accumulate == 0) or rhs += v + s.  Arguments and
 * layouts as for sem_volume_rhs, plus nbr [Ne][6] as for sem_surface_rhs
 * (conforming aligned faces; a neighbour index outside [0, Ne) is a boundary
 * face that adds nothing).  The result equals sem_volume_rhs followed by
 * sem_surface_rhs with accumulate up to rounding (the face terms join the
 * sum before the 1/J scaling).
 * Nq: 2..10.
 * No byte of rhs may lie inside an input (D, geo, q, rho_ref, theta_ref, nbr).
 * Errors: as for sem_volume_rhs; NULL or misaligned nbr -> SEM_ERR_INVALID_ARG.
 * Allocates nothing; enqueues one kernel launch. */
sem_status sem_rhs(int32_t Ne, int32_t Nq, sem_dtype dtype, const void* D, const void* geo,
                   const void* q, const void* rho_ref, const double* theta_ref,
                   const int32_t* nbr, const sem_phys* phys, void* rhs, int32_t accumulate,
                   void* stream);

/* out[i] = a*x[i] + b*(y[i] + c*z[i]) for i < n (x may be NULL when a == 0):
 * the stage update of an explicit Runge-Kutta method for the method-of-lines
 * system dq/dt = v(q) + s(q) of Sec. 2 (with y the stage state, z its rate
 * and c the time step).  out may be the same array as x, y or z; a partial
 * overlap (same memory at a different index) is rejected.  Arrays aligned to
 * 16 bytes run vector accesses, others a scalar path with the same results.
 * Errors: n < 0, NULL required pointer, misalignment, partial overlap ->
 * SEM_ERR_INVALID_ARG.  Allocates nothing. */
sem_status sem_axpby(int64_t n, sem_dtype dtype, double a, const void* x, double b,
                     const void* y, double c, const void* z, void* out, void* stream);

/* ---------------------------------------------------------------------------
 * Mixed-order batch: many element blocks, each of one order, evaluated by ONE
 * kernel launch (one tile of elements per workgroup).  The volume term of
 * Eq. (volterm) is local to an element (Sec. 2 evaluates it element by
 * element, the listed kernels loop over e), so blocks of different polynomial
 * order are independent and share one launch.  A block has the layouts above
 * with its own Nq and Ne; every block of a plan shares dtype and phys.
 * ------------------------------------------------------------------------- */
typedef struct sem_block {
    int32_t Nq;
    int32_t Ne;
    const void* D;
    const void* geo;
    const void* q;
    const void* rho_ref;       /* nullable */
    const double* theta_ref;   /* nullable, FP64 */
    void* rhs;
} sem_block;

typedef struct sem_plan_s* sem_plan;

#define SEM_PLAN_AUTOTUNE 1u   /* time candidate tile shapes on the device (synchronises;
                                  the timing launches write the blocks' rhs arrays) */
#define SEM_PLAN_USE_CACHE 2u  /* read/write tuned shapes in the JSON file named by the
                                  SEM_PLAN_CACHE environment variable (ignored if unset) */

/* Builds a plan: picks a tile shape per order (autotuned or default), orders
 * the tiles longest-first and uploads a device tile table owned by the plan.
 * One launch has one workgroup size and one LDS size (its largest shape's);
 * the autotuner times every order's candidate shapes at each possible LDS
 * size and keeps the combination with the smallest total time.
 * The block pointers are baked in: the caller keeps those buffers alive and
 * unchanged in address for the plan's lifetime.  Errors: nblocks < 1, any
 * invalid block (as sem_volume_rhs), SEM_ERR_NO_MEMORY, SEM_ERR_HIP. */
sem_status sem_batch_plan(const sem_block* blocks, int32_t nblocks, sem_dtype dtype,
                          const sem_phys* phys, uint32_t flags, void* stream,
                          sem_plan* out);

/* Enqueues the whole batch as one launch: rhs of every block =
 * v(q) of that block.  Allocates nothing and records only the kernel launch,
 * so a caller may capture it into a HIP graph. */
sem_status sem_batch_execute(sem_plan plan, void* stream);

/* Writes a JSON description of the plan's choices (NUL-terminated, truncated
 * to len).  Returns SEM_ERR_INVALID_ARG for a NULL plan or buffer. */
sem_status sem_plan_describe(sem_plan plan, char* buf, int32_t len);

/* Frees the plan and its device tables (after the enqueued work finished). */
sem_status sem_plan_destroy(sem_plan plan);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * mixed-order batch of sem_batch_plan + sem_batch_execute in one call that
 * allocates nothing.
 *
 * rhs of every block = v(q) (overwrite), evaluated with the built-in tile
 * shapes (those of sem_batch_plan without SEM_PLAN_AUTOTUNE; the results are
 * the same bit for bit).  Enqueues two kernel launches on `stream`: one that
 * writes the tile and block tables into a device array of the library
 * (SEM_STATIC_MAX_BLOCKS block descriptors and SEM_STATIC_MAX_TILES tiles,
 * 770 KiB, held on each GPU the library runs on until the process ends), and
 * the batch kernel.  No hipMalloc, hipFree, copy or memset; nothing to reset
 * between calls (the tables are rewritten by every call).
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (on different streams, or from several threads without ordering) race.
 * Blocks, layouts and checks as for sem_batch_plan; the caller keeps the
 * arrays alive until the launch has run.
 * Errors: as sem_batch_plan, plus nblocks > SEM_STATIC_MAX_BLOCKS or more than
 * SEM_STATIC_MAX_TILES tiles -> SEM_ERR_INVALID_ARG.
 * ------------------------------------------------------------------------- */
#define SEM_STATIC_MAX_BLOCKS 16
#define SEM_STATIC_MAX_TILES 32768

sem_status sem_batch_rhs_static(const sem_block* blocks, int32_t nblocks, sem_dtype dtype,
                                const sem_phys* phys, void* stream);

/* ---------------------------------------------------------------------------
 * One SSP-RK3 (Shu-Osher) step of dq/dt = v(q) (explicit time integration of
 * the method-of-lines rate, Sec. 2), captured once in a HIP graph:
 *   q1 = q + dt v(q);  q2 = 3/4 q + 1/4 (q1 + dt v(q1));
 *   q  = 1/3 q + 2/3 (q2 + dt v(q2))          (q updated in place)
 * By default each stage is ONE batch launch whose epilogue writes
 * the stage update directly (the rate is never stored).  With
 * SEM_RK3_SEPARATE_STAGES each stage is a batch launch writing v into L plus
 * one sem_axpby.
 * q_n, q_1, q_2, L are distinct flat buffers of n values of dtype.  The
 * blocks' q arrays must tile q_n[0, n) exactly (no gap, no overlap), and each
 * block's rhs must sit in L at the offset of its q in q_n (the stage plans
 * read q_1 and q_2 at that offset); otherwise SEM_ERR_INVALID_ARG.  L is
 * written only with SEM_RK3_SEPARATE_STAGES (then it holds the last stage's
 * rate).
 * flags: SEM_PLAN_AUTOTUNE / SEM_PLAN_USE_CACHE (tile shapes, chosen once and
 * shared by the three stages) and SEM_RK3_SEPARATE_STAGES.
 * ------------------------------------------------------------------------- */
typedef struct sem_rk3_s* sem_rk3;

#define SEM_RK3_SEPARATE_STAGES 4u

sem_status sem_rk3_graph_create(const sem_block* blocks, int32_t nblocks, sem_dtype dtype,
                                const sem_phys* phys, uint32_t flags, void* q_n, void* q_1,
                                void* q_2, void* L, int64_t n, double dt, void* stream,
                                sem_rk3* out);

/* Launches the captured step on `stream`.  Allocates nothing. */
sem_status sem_rk3_graph_launch(sem_rk3 step, void* stream);

/* Writes a JSON description (stage mode and the shared stage plan). */
sem_status sem_rk3_graph_describe(sem_rk3 step, char* buf, int32_t len);

/* Frees the graph and its three stage plans. */
sem_status sem_rk3_graph_destroy(sem_rk3 step);

#ifdef __cplusplus
}
#endif

#endif /* SEMVOL_SEM_H */
