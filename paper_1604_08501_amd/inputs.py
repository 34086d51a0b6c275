"""Seeded synthetic inputs for the strong-form spectral-element volume term.

This module builds everything the volume term takes as *input*: the
Gauss-Lobatto-Legendre (GLL) nodes and the nodal differentiation matrix D,
hexahedral meshes with their per-node metric terms g and inverse Jacobian,
a random prognostic state, a hydrostatic reference state, cotangents and
finite-difference directions.  It deliberately contains none of the volume
term's own arithmetic (no flux, no equation of state, no contraction): both
the HIP path and the CPU oracle consume the arrays produced here, and they
share nothing else.

Conventions (Sec. 2 of the paper, Eq. (volterm) and Fig. 1):

* node index inside an element ``m = i + Nq*j + Nq^2*k``; ``i, j, k`` run along
  the reference directions ``r, s, t``;
* state ``q[e][5][Nq^3]`` with the fields in the order of the prognostic
  vector: rho, U1 = rho*u, U2 = rho*v, U3 = rho*w, Theta = rho*theta;
* geometry ``geo[e][10][Nq^3]``: slot ``3*d + a`` (``a, d`` in 0..2) holds
  ``g_{a d} = J * d xi_d / d x_a`` (the cofactor of ``A = dx/dxi``), slot 9
  holds ``1/J``;
* ``D[i*Nq + n] = l_n'(xi_i)`` (row = output node).

Every random draw comes from ``numpy.random.default_rng(160408501 + k)`` in a
fixed order, so a configuration is reproducible from its index ``k``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_BASE = 160408501

# Physical constants of the synthetic workloads (p0 in Pa, R in J/(kg K),
# g in m/s^2).  The paper's own benchmark fixes p0 = 1, gamma = 1.4, R = 1
# and leaves gravity out; the workloads here use atmospheric values.
P0 = 1.0e5
GAMMA = 1.4
R_GAS = 287.0
GRAV = 9.81
THETA0 = 300.0      # reference potential temperature, K
RHO_SURF = 1.0      # reference density at z = 0, kg/m^3
LENGTH = 1000.0     # edge of the warped box, m
WARP = 0.05         # amplitude of the sine warp (unit-cube coordinates)

NFIELDS = 5
NGEO = 10


# --------------------------------------------------------------------------
# GLL nodes, weights and the differentiation matrix
# --------------------------------------------------------------------------
def _legendre(N: int, x: np.ndarray):
    """Return (P_N(x), P_N'(x)) by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if N == 0:
        return p_prev, np.zeros_like(x)
    p = x.copy()
    dp_prev = np.zeros_like(x)
    dp = np.ones_like(x)
    for n in range(2, N + 1):
        p_next = ((2 * n - 1) * x * p - (n - 1) * p_prev) / n
        dp_next = dp_prev + (2 * n - 1) * p
        p_prev, p = p, p_next
        dp_prev, dp = dp, dp_next
    return p, dp


def gll_nodes(N: int) -> np.ndarray:
    """GLL points for polynomial order N: -1, the N-1 roots of P_N', +1.

    Newton's method on ``q(x) = P_{N+1}(x) - P_{N-1}(x)``, which is a multiple
    of ``(1 - x^2) P_N'(x)`` and has derivative ``(2N + 1) P_N(x)``, started
    from the Chebyshev-Gauss-Lobatto points.  Symmetry is imposed at the end.
    """
    if N < 1:
        raise ValueError("N >= 1 required")
    x = -np.cos(np.pi * np.arange(N + 1) / N)
    for _ in range(100):
        pNp1, _ = _legendre(N + 1, x)
        pNm1, _ = _legendre(N - 1, x)
        pN, _ = _legendre(N, x)
        dx = (pNp1 - pNm1) / ((2 * N + 1) * pN)
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    x[0], x[-1] = -1.0, 1.0
    x = 0.5 * (x - x[::-1])
    if N % 2 == 0:
        x[N // 2] = 0.0
    return x


def gll_weights(N: int) -> np.ndarray:
    """GLL quadrature weights ``2 / (N (N+1) P_N(x_j)^2)``."""
    x = gll_nodes(N)
    pN, _ = _legendre(N, x)
    return 2.0 / (N * (N + 1) * pN ** 2)


def diff_matrix(N: int) -> np.ndarray:
    """Nodal differentiation matrix on the GLL points, ``D[i, n] = l_n'(x_i)``.

    Off-diagonal entries from the barycentric form of the Lagrange basis,
    ``(w_n / w_i) / (x_i - x_n)`` with ``w_j = 1 / prod_{k != j}(x_j - x_k)``;
    the diagonal by the negative-sum trick so that every row sum is zero
    (D annihilates constants to round-off).
    """
    x = gll_nodes(N)
    n = N + 1
    diff = x[:, None] - x[None, :]
    np.fill_diagonal(diff, 1.0)
    w = 1.0 / np.prod(diff, axis=1)
    D = (w[None, :] / w[:, None]) / diff
    np.fill_diagonal(D, 0.0)
    D[np.arange(n), np.arange(n)] = -D.sum(axis=1)
    return D


# --------------------------------------------------------------------------
# Meshes and metric terms
# --------------------------------------------------------------------------
def _cofactor_jac(A: np.ndarray):
    """For ``A[..., a, d] = dx_a/dxi_d`` return ``(g, J)`` with
    ``g[..., a, d] = cof(A)[a, d] = J * dxi_d/dx_a`` and ``J = det A``."""
    a = A
    c = np.empty_like(a)
    c[..., 0, 0] = a[..., 1, 1] * a[..., 2, 2] - a[..., 1, 2] * a[..., 2, 1]
    c[..., 0, 1] = a[..., 1, 2] * a[..., 2, 0] - a[..., 1, 0] * a[..., 2, 2]
    c[..., 0, 2] = a[..., 1, 0] * a[..., 2, 1] - a[..., 1, 1] * a[..., 2, 0]
    c[..., 1, 0] = a[..., 0, 2] * a[..., 2, 1] - a[..., 0, 1] * a[..., 2, 2]
    c[..., 1, 1] = a[..., 0, 0] * a[..., 2, 2] - a[..., 0, 2] * a[..., 2, 0]
    c[..., 1, 2] = a[..., 0, 1] * a[..., 2, 0] - a[..., 0, 0] * a[..., 2, 1]
    c[..., 2, 0] = a[..., 0, 1] * a[..., 1, 2] - a[..., 0, 2] * a[..., 1, 1]
    c[..., 2, 1] = a[..., 0, 2] * a[..., 1, 0] - a[..., 0, 0] * a[..., 1, 2]
    c[..., 2, 2] = a[..., 0, 0] * a[..., 1, 1] - a[..., 0, 1] * a[..., 1, 0]
    J = (a[..., 0, 0] * c[..., 0, 0] + a[..., 0, 1] * c[..., 0, 1]
         + a[..., 0, 2] * c[..., 0, 2])
    return c, J


def pack_geo(A: np.ndarray) -> np.ndarray:
    """Pack per-node Jacobian matrices ``A[e, m, a, d]`` into ``geo[e][10][m]``."""
    g, J = _cofactor_jac(A)
    Ne, M = A.shape[:2]
    geo = np.empty((Ne, NGEO, M), dtype=np.float64)
    for d in range(3):
        for a in range(3):
            geo[:, 3 * d + a, :] = g[..., a, d]
    geo[:, 9, :] = 1.0 / J
    return geo


def _ref_coords(N: int):
    """Reference coordinates of the Nq^3 nodes, each shaped (Nq^3,), i fastest."""
    x = gll_nodes(N)
    Nq = N + 1
    m = np.arange(Nq ** 3)
    return x[m % Nq], x[(m // Nq) % Nq], x[m // (Nq * Nq)]


def _nodal_derivative(D: np.ndarray, F: np.ndarray, d: int) -> np.ndarray:
    """Apply the 1-D differentiation matrix along reference direction d to
    nodal fields F[..., m] (m = i + Nq j + Nq^2 k)."""
    Nq = D.shape[0]
    G = F.reshape(F.shape[:-1] + (Nq, Nq, Nq))       # [..., k, j, i]
    if d == 0:
        out = np.einsum("in,...kjn->...kji", D, G)
    elif d == 1:
        out = np.einsum("jn,...kni->...kji", D, G)
    else:
        out = np.einsum("kn,...nji->...kji", D, G)
    return out.reshape(F.shape)


def curl_metric_geo(xyz: np.ndarray, N: int) -> np.ndarray:
    """Metric terms in conservative curl form from the nodal coordinates
    ``xyz[e][3][Nq^3]``: for cyclic (d, e, f) and cyclic (a, b, c)

        g_ad = D_f (x_c D_e x_b) - D_e (x_c D_f x_b),

    the discrete counterpart of J dxi_d/dx_a = (dx/dxi_e x dx/dxi_f)_a.  Since
    the tensor-product derivatives commute, sum_d D_d g_ad = 0 holds to round-off
    (the discrete metric identities), so a uniform state keeps a zero flux
    divergence on curved elements.  1/J comes from the determinant of the
    discrete Jacobian D_d x_a.
    """
    D = diff_matrix(N)
    Ne, _, M = xyz.shape
    # the curl form is unchanged by a translation of x (the derivatives
    # commute); element-local coordinates keep the products small
    xyz = xyz - xyz.mean(axis=2, keepdims=True)
    dx = np.stack([_nodal_derivative(D, xyz, d) for d in range(3)], axis=-1)   # [e, a, m, d]
    geo = np.empty((Ne, NGEO, M))
    for d in range(3):
        e_, f_ = (d + 1) % 3, (d + 2) % 3
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            Pe = xyz[:, c] * dx[:, b, :, e_]
            Pf = xyz[:, c] * dx[:, b, :, f_]
            geo[:, 3 * d + a] = _nodal_derivative(D, Pe, f_) - _nodal_derivative(D, Pf, e_)
    A = dx.transpose(0, 2, 1, 3)                                          # [e, m, a, d]
    _, J = _cofactor_jac(A)
    geo[:, 9] = 1.0 / J
    return geo


def box_neighbours(n_side, elements: Optional[np.ndarray] = None) -> np.ndarray:
    """Face neighbours of the structured box of ``nx x ny x nz`` elements
    ``e = ex + nx (ey + ny ez)``, periodic in every direction: ``nbr[e][f]``
    for the faces f = r-, r+, s-, s+, t-, t+ (reference direction d = f // 2,
    side f % 2), an int32 ``[Ne, 6]`` array indexing ``elements``.  A
    neighbour outside the ``elements`` subset is ``-1`` (a boundary face).
    Neighbouring elements of the box share the face with aligned node
    numbering: node (0, j, k) of an element meets node (N, j, k) of the one
    across its r = -1 face."""
    nx, ny, nz = (n_side,) * 3 if np.isscalar(n_side) else tuple(n_side)
    if elements is None:
        elements = np.arange(nx * ny * nz)
    elements = np.asarray(elements, dtype=np.int64)
    pos = np.full(nx * ny * nz, -1, dtype=np.int64)
    pos[elements] = np.arange(elements.size)
    ex = elements % nx
    ey = (elements // nx) % ny
    ez = elements // (nx * ny)
    nbr = np.empty((elements.size, 6), dtype=np.int32)
    for f, (dx, dy, dz) in enumerate(((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0),
                                      (0, 0, -1), (0, 0, 1))):
        g = (ex + dx) % nx + nx * ((ey + dy) % ny + ny * ((ez + dz) % nz))
        nbr[:, f] = pos[g]
    return nbr


@dataclasses.dataclass
class Mesh:
    N: int
    Ne: int
    geo: np.ndarray        # (Ne, 10, Nq^3) float64
    xyz: np.ndarray        # (Ne, 3, Nq^3) float64 physical node coordinates
    A: np.ndarray          # (Ne, Nq^3, 3, 3) float64, dx_a/dxi_d
    kind: str

    @property
    def Nq(self) -> int:
        return self.N + 1


def affine_mesh(N: int, rng: np.random.Generator, n_side: int = 4) -> Mesh:
    """``n_side^3`` affine elements ``x = A_e xi + b_e``.

    ``A_e = I + 0.1 U(-1, 1)^{3x3}`` (one draw per element, element order
    ``e = ex + n(ey + n ez)``), ``b_e = 2 (ex, ey, ez) + 1``.  By Gershgorin
    every ``det A_e > 0``.
    """
    Ne = n_side ** 3
    Ae = np.eye(3)[None] + 0.1 * rng.uniform(-1.0, 1.0, size=(Ne, 3, 3))
    e = np.arange(Ne)
    b = 2.0 * np.stack([e % n_side, (e // n_side) % n_side, e // (n_side * n_side)], axis=1) + 1.0
    r, s, t = _ref_coords(N)
    xi = np.stack([r, s, t], axis=0)                     # (3, M)
    xyz = np.einsum("ead,dm->eam", Ae, xi) + b[:, :, None]
    M = xi.shape[1]
    A = np.broadcast_to(Ae[:, None], (Ne, M, 3, 3)).copy()
    return Mesh(N=N, Ne=Ne, geo=pack_geo(A), xyz=xyz, A=A, kind="affine")


def warped_mesh(N: int, n_side=32, elements: Optional[np.ndarray] = None,
                length=LENGTH, warp: float = WARP, metrics: str = "analytic") -> Mesh:
    """Curvilinear box: ``n_side^3`` elements of the unit cube (or
    ``nx x ny x nz`` when ``n_side`` is a triple), warped by

        x += w sin(pi y) sin(pi z),  y += w sin(pi z) sin(pi x),
        z += w sin(pi x) sin(pi y)

    (all three applied simultaneously to the unwarped unit-cube coordinates),
    then scaled by ``length`` (a number, or one length per axis).  Metric terms
    come from the analytic derivative of the map at every node.  ``elements``
    selects a subset of the element indices ``e = ex + nx(ey + ny ez)``
    (default: all).  ``metrics="curl"`` forms the metric terms in
    conservative curl form from the node coordinates (see
    :func:`curl_metric_geo`) instead of the analytic Jacobian.
    """
    if metrics not in ("analytic", "curl"):
        raise ValueError("metrics must be 'analytic' or 'curl'")
    nx, ny, nz = (n_side,) * 3 if np.isscalar(n_side) else tuple(n_side)
    Lx, Ly, Lz = (length,) * 3 if np.isscalar(length) else tuple(length)
    if elements is None:
        elements = np.arange(nx * ny * nz)
    elements = np.asarray(elements, dtype=np.int64)
    Ne = elements.size
    r, s, t = _ref_coords(N)
    ex = elements % nx
    ey = (elements // nx) % ny
    ez = elements // (nx * ny)
    X = (ex[:, None] + 0.5 * (r[None] + 1.0)) / nx
    Y = (ey[:, None] + 0.5 * (s[None] + 1.0)) / ny
    Z = (ez[:, None] + 0.5 * (t[None] + 1.0)) / nz
    pi = np.pi
    sx, cx = np.sin(pi * X), np.cos(pi * X)
    sy, cy = np.sin(pi * Y), np.cos(pi * Y)
    sz, cz = np.sin(pi * Z), np.cos(pi * Z)
    xh = X + warp * sy * sz
    yh = Y + warp * sz * sx
    zh = Z + warp * sx * sy
    # dxhat_a / dX_b
    M = X.shape[1]
    Ah = np.zeros((Ne, M, 3, 3))
    Ah[..., 0, 0] = 1.0
    Ah[..., 0, 1] = warp * pi * cy * sz
    Ah[..., 0, 2] = warp * pi * sy * cz
    Ah[..., 1, 0] = warp * pi * sz * cx
    Ah[..., 1, 1] = 1.0
    Ah[..., 1, 2] = warp * pi * cz * sx
    Ah[..., 2, 0] = warp * pi * cx * sy
    Ah[..., 2, 1] = warp * pi * sx * cy
    Ah[..., 2, 2] = 1.0
    # x_a = L_a xhat_a, dX_b / dxi_d = delta_bd / (2 n_b)
    Lv = np.array([Lx, Ly, Lz])
    nv = np.array([nx, ny, nz], dtype=np.float64)
    A = Ah * Lv[:, None] * (0.5 / nv)[None, :]
    xyz = np.stack([Lx * xh, Ly * yh, Lz * zh], axis=1)
    geo = pack_geo(A) if metrics == "analytic" else curl_metric_geo(xyz, N)
    return Mesh(N=N, Ne=Ne, geo=geo, xyz=xyz, A=A, kind="warped" if metrics == "analytic"
                else "warped-curl")


# --------------------------------------------------------------------------
# Reference state and random prognostic state
# --------------------------------------------------------------------------
def hydrostatic_reference(z: np.ndarray, p0: float = P0, gamma: float = GAMMA,
                          R: float = R_GAS, grav: float = GRAV,
                          theta0: float = THETA0, rho_s: float = RHO_SURF):
    """Isentropic hydrostatic profile with constant potential temperature.

    Exner function ``pi(z) = pi_s - g z / (c_p theta0)`` with
    ``pi_s = (R rho_s theta0 / p0)^(gamma - 1)`` and ``c_p = gamma R/(gamma-1)``;
    ``p_ref = p0 pi^(c_p/R)``, ``rho_ref = p_ref / (R pi theta0)``,
    ``Theta_ref = rho_ref theta0``.  Returns ``(rho_ref, Theta_ref, p_ref)``.
    """
    cp = gamma * R / (gamma - 1.0)
    pi_s = (R * rho_s * theta0 / p0) ** (gamma - 1.0)
    ex = pi_s - grav * z / (cp * theta0)
    p_ref = p0 * ex ** (cp / R)
    rho_ref = p_ref / (R * ex * theta0)
    return rho_ref, rho_ref * theta0, p_ref


@dataclasses.dataclass
class Phys:
    p0: float = P0
    gamma: float = GAMMA
    R: float = R_GAS
    grav: float = GRAV

    def as_tuple(self):
        return (self.p0, self.gamma, self.R, self.grav)


def random_state(rng: np.random.Generator, Ne: int, Nq: int) -> np.ndarray:
    """``rho = 1 + 0.01 N(0,1)``, ``U = rho * 10 N(0,1)`` per component,
    ``Theta = rho (300 + N(0,1))``; draws in the order rho-noise, u, v, w,
    theta-noise, each shaped ``(Ne, Nq^3)``."""
    M = Nq ** 3
    rho = 1.0 + 0.01 * rng.standard_normal((Ne, M))
    u = 10.0 * rng.standard_normal((Ne, M))
    v = 10.0 * rng.standard_normal((Ne, M))
    w = 10.0 * rng.standard_normal((Ne, M))
    th = 300.0 + rng.standard_normal((Ne, M))
    q = np.empty((Ne, NFIELDS, M))
    q[:, 0] = rho
    q[:, 1] = rho * u
    q[:, 2] = rho * v
    q[:, 3] = rho * w
    q[:, 4] = rho * th
    return q


FD_SCALES = (0.01, 10.0, 10.0, 10.0, 3.0)


@dataclasses.dataclass
class Workload:
    """One synthetic workload: mesh, D, state, reference state, constants."""
    name: str
    N: int
    D: np.ndarray           # (Nq, Nq) float64
    geo: np.ndarray         # (Ne, 10, Nq^3) float64
    q: np.ndarray           # (Ne, 5, Nq^3) float64
    rho_ref: np.ndarray     # (Ne, Nq^3) float64
    theta_ref: np.ndarray   # (Ne, Nq^3) float64
    phys: Phys
    xyz: np.ndarray
    lam: Optional[np.ndarray] = None    # cotangent (Ne, 5, Nq^3)
    dq: Optional[np.ndarray] = None     # FD direction (Ne, 5, Nq^3)
    nbr: Optional[np.ndarray] = None    # face neighbours (Ne, 6) int32, box meshes only

    @property
    def Nq(self) -> int:
        return self.N + 1

    @property
    def Ne(self) -> int:
        return self.q.shape[0]


def _finish(name, N, mesh, rng, with_adjoint) -> Workload:
    Nq = N + 1
    q = random_state(rng, mesh.Ne, Nq)
    rho_ref, theta_ref, _ = hydrostatic_reference(mesh.xyz[:, 2, :])
    lam = dq = None
    if with_adjoint:
        lam = rng.standard_normal(q.shape)
        dq = rng.standard_normal(q.shape) * np.asarray(FD_SCALES)[None, :, None]
    return Workload(name=name, N=N, D=diff_matrix(N), geo=mesh.geo, q=q,
                    rho_ref=rho_ref, theta_ref=theta_ref, phys=Phys(),
                    xyz=mesh.xyz, lam=lam, dq=dq)


def affine_workload(N: int = 4, n_side: int = 4, k: int = 1,
                    with_adjoint: bool = True) -> Workload:
    """Plain affine workload: N=4 on 4x4x4 random affine hexahedra (seed k=1)."""
    rng = np.random.default_rng(SEED_BASE + k)
    mesh = affine_mesh(N, rng, n_side)
    return _finish(f"affine_N{N}_Ne{mesh.Ne}", N, mesh, rng, with_adjoint)


def warped_workload(N: int = 7, n_side: int = 32, n_elements: Optional[int] = None,
                    k: int = 2, with_adjoint: bool = False, metrics: str = "analytic") -> Workload:
    """Warped-box workload: the first ``n_elements`` elements (default all
    ``n_side^3``) of the warped ``n_side^3`` box at order N (seed k)."""
    rng = np.random.default_rng(SEED_BASE + k)
    total = n_side ** 3
    n = total if n_elements is None else int(n_elements)
    mesh = warped_mesh(N, n_side, np.arange(n), metrics=metrics)
    w = _finish(f"warped_N{N}_Ne{n}", N, mesh, rng, with_adjoint)
    w.nbr = box_neighbours(n_side, np.arange(n))
    return w


def mixed_order_workloads(orders=(3, 5, 7, 9), per_order: int = 5000, k: int = 3):
    """Mixed-order batch: for each order the first ``per_order`` elements of
    the warped 32^3 box, each order with its own seeded state (one generator,
    drawn order by order)."""
    rng = np.random.default_rng(SEED_BASE + k)
    out = []
    for N in orders:
        mesh = warped_mesh(N, 32, np.arange(per_order))
        out.append(_finish(f"warped_N{N}_Ne{per_order}", N, mesh, rng, False))
    return out


def adjoint_workload(N: int = 7, n_elements: int = 8192, k: int = 5) -> Workload:
    """Adjoint workload: the first 8192 warped elements at N=7, with a
    cotangent lambda ~ N(0,1) and an FD direction (seed k=5)."""
    rng = np.random.default_rng(SEED_BASE + k)
    mesh = warped_mesh(N, 32, np.arange(n_elements))
    return _finish(f"adjoint_N{N}_Ne{n_elements}", N, mesh, rng, True)


def element_geo(geo: np.ndarray) -> np.ndarray:
    """Per-element metric terms ``[Ne][10]`` of an affine mesh (whose per-node
    terms ``geo[e][10][Nq^3]`` are constant in each element)."""
    g = np.ascontiguousarray(geo[:, :, 0])
    if np.max(np.ptp(geo, axis=2)) > 1e-12 * np.max(np.abs(geo)):
        raise ValueError("metric terms vary inside an element: not an affine mesh")
    return g


def add_tracers(w: Workload, k: int = 100) -> Workload:
    """The same workload with three passive tracers appended to the state:
    ``Q_i = rho (0.2 i + 0.5 + 0.05 N(0,1))`` (seeded by ``k`` on a generator of
    its own, so the other fields are unchanged)."""
    rng = np.random.default_rng(SEED_BASE + k)
    rho = w.q[:, :1]
    Q = rho * (0.2 * np.arange(1, 4)[None, :, None] + 0.5
               + 0.05 * rng.standard_normal((w.Ne, 3, w.q.shape[2])))
    return dataclasses.replace(w, q=np.ascontiguousarray(np.concatenate([w.q, Q], axis=1)),
                               name=w.name + "_tracers")


# The paper's Table 2 keeps 3,538,944 nodes while Nq varies: Ne = 55296, 6912,
# 2048, 864 at Nq = 4, 8, 12, 16 are the elements of a 2:2:1 box of
# 192 x 192 x 96 nodes (nz = 96 / Nq elements vertically).
TABLE2_NODES = 3538944


def table2_workload(Nq: int, k: int = 7, tracers: bool = True) -> Workload:
    """Warped 2 km x 2 km x 1 km box with (2 nz, 2 nz, nz) elements,
    nz = 96 / Nq, i.e. the paper's constant 3,538,944-node workload."""
    if 96 % Nq:
        raise ValueError("Nq must divide 96 (Table 2 uses Nq = 4, 8, 12, 16)")
    nz = 96 // Nq
    rng = np.random.default_rng(SEED_BASE + k)
    mesh = warped_mesh(Nq - 1, (2 * nz, 2 * nz, nz), length=(2 * LENGTH, 2 * LENGTH, LENGTH))
    w = _finish(f"table2_Nq{Nq}_Ne{mesh.Ne}", Nq - 1, mesh, rng, False)
    return add_tracers(w, 100 + k) if tracers else w


def to_fp32(w: Workload) -> Workload:
    """Round every array of a workload to FP32 storage except Theta_ref,
    which stays FP64; the FP32 values are returned as float32 arrays."""
    f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
    return dataclasses.replace(
        w, D=f(w.D), geo=f(w.geo), q=f(w.q), rho_ref=f(w.rho_ref),
        theta_ref=np.ascontiguousarray(w.theta_ref, dtype=np.float64),
        lam=f(w.lam), dq=f(w.dq))


def upcast(w: Workload) -> Workload:
    """Exact FP64 copy of a (possibly FP32-rounded) workload."""
    f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    return dataclasses.replace(w, D=f(w.D), geo=f(w.geo), q=f(w.q),
                               rho_ref=f(w.rho_ref), theta_ref=f(w.theta_ref),
                               lam=f(w.lam), dq=f(w.dq))


def rel_err_per_field(out: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """``max|out_b - ref_b| / max|ref_b|`` for every field b (axis 1)."""
    out = np.asarray(out, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    nf = ref.shape[1]
    num = np.abs(out - ref).transpose(1, 0, 2).reshape(nf, -1).max(axis=1)
    den = np.abs(ref).transpose(1, 0, 2).reshape(nf, -1).max(axis=1)
    return num / np.where(den > 0, den, 1.0)
