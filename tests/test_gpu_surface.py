"""GPU parity of the surface term (the s of dq/dt = v + s: strong-form
discontinuous Galerkin face term with a local Lax-Friedrichs flux) through the
C-ABI, against the CPU oracle element by element.

Gates as for the volume term: FP64 <= 1e-12, FP32 <= 2e-5 (oracle on the
FP32-rounded inputs, upcast exactly, with the shared FP64 Theta_ref), max
relative error per field normalised by max|oracle| of that field.
"""
import numpy as np
import pytest
import torch

from paper_1604_08501_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 2e-5


@pytest.fixture(scope="module")
def sv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_08501_amd as m
    m.lib()
    return m


def dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def err(out, ref):
    return I.rel_err_per_field(out, ref)


def run(sv, w, nbr=None, with_ref=True, out=None, accumulate=False, fp32=False):
    src = I.to_fp32(w) if fp32 else w
    return sv.surface_rhs(dev(src.q), dev(src.geo), dev(w.nbr if nbr is None else nbr),
                          dev(w.theta_ref) if with_ref else None, w.phys.as_tuple(), out=out,
                          accumulate=accumulate)


def oracle_s(oracle_mod, w, nbr=None, with_ref=True, fp32=False):
    src = I.upcast(I.to_fp32(w)) if fp32 else w
    return oracle_mod.surface_rhs(src.geo, src.q, w.nbr if nbr is None else nbr,
                                  w.theta_ref if with_ref else None, w.phys.as_tuple())


@pytest.mark.parametrize("Nq", [2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 16])
def test_surface_vs_oracle(sv, oracle_mod, Nq):
    """Every order on a periodic warped box (3^3 elements, 2^3 at Nq >= 12):
    FP64 and FP32, with and without the reference state, overwrite and
    accumulate."""
    n_side = 3 if Nq <= 10 else 2
    w = I.warped_workload(N=Nq - 1, n_side=n_side, k=300 + Nq)
    for with_ref in (True, False):
        ref = oracle_s(oracle_mod, w, with_ref=with_ref)
        e = err(host(run(sv, w, with_ref=with_ref)), ref)
        assert e.max() <= TOL64, (Nq, with_ref, e)
        base = np.random.default_rng(Nq).standard_normal(w.q.shape)
        out = dev(base.copy())
        run(sv, w, with_ref=with_ref, out=out, accumulate=True)
        assert err(host(out), base + ref).max() <= TOL64, (Nq, with_ref)
        ref32 = oracle_s(oracle_mod, w, with_ref=with_ref, fp32=True)
        e32 = err(host(run(sv, w, with_ref=with_ref, fp32=True)), ref32)
        assert e32.max() <= TOL32, (Nq, with_ref, e32)
        b32 = base.astype(np.float32)
        out32 = dev(b32.copy())
        run(sv, w, with_ref=with_ref, out=out32, accumulate=True, fp32=True)
        assert err(host(out32), b32.astype(np.float64) + ref32).max() <= TOL32, (Nq, with_ref)


def test_surface_boundary_faces_and_out_of_range_neighbours(sv, oracle_mod):
    """A mesh cut out of the box (neighbours outside it are -1) with some
    indices set beyond Ne or below -1: every such face is a boundary face and
    adds nothing, exactly as in the oracle; the kernel reads nothing through
    them."""
    w = I.warped_workload(N=4, n_side=4, n_elements=21, k=320)
    nbr = w.nbr.copy()
    nbr[3, 1] = w.Ne + 5
    nbr[7, 4] = 2 ** 31 - 1
    nbr[11, 2] = -7
    assert (nbr < 0).any()
    ref = oracle_s(oracle_mod, w, nbr=nbr)
    assert err(host(run(sv, w, nbr=nbr)), ref).max() <= TOL64
    ref32 = oracle_s(oracle_mod, w, nbr=nbr, fp32=True)
    assert err(host(run(sv, w, nbr=nbr, fp32=True)), ref32).max() <= TOL32
    none = np.full_like(w.nbr, -1)
    assert np.all(host(run(sv, w, nbr=none)) == 0.0)


def test_single_element_periodic_onto_itself(sv, oracle_mod):
    """One element whose six neighbours are itself (a 1^3 periodic box)."""
    w = I.warped_workload(N=5, n_side=1, k=321)
    assert np.all(w.nbr == 0)
    assert err(host(run(sv, w)), oracle_s(oracle_mod, w)).max() <= TOL64
    assert err(host(run_rhs(sv, w)), oracle_vs(oracle_mod, w)).max() <= TOL64


def test_volume_plus_surface_is_conservative(sv, oracle_mod):
    """sem_volume_rhs then sem_surface_rhs with accumulate gives v + s; on the
    periodic box its GLL quadrature of J (v + s) vanishes (no source), as the
    oracle's does."""
    N = 4
    w = I.warped_workload(N=N, n_side=4, k=322)
    phys = (I.P0, I.GAMMA, I.R_GAS, 0.0)
    q, geo, D, rr, tr = dev(w.q), dev(w.geo), dev(w.D), dev(w.rho_ref), dev(w.theta_ref)
    out = sv.volume_rhs(q, geo, D, rr, tr, phys)
    sv.surface_rhs(q, geo, dev(w.nbr), tr, phys, out=out, accumulate=True)
    got = host(out)
    ref = oracle_mod.volume_rhs(w.D, w.geo, w.q, w.rho_ref, w.theta_ref, phys) + \
        oracle_mod.surface_rhs(w.geo, w.q, w.nbr, w.theta_ref, phys)
    assert err(got, ref).max() <= TOL64
    wq = I.gll_weights(N)
    Nq = N + 1
    m = np.arange(Nq ** 3)
    W = (wq[m % Nq] * wq[(m // Nq) % Nq] * wq[m // (Nq * Nq)])[None, :] / w.geo[:, 9]
    tot = np.einsum("em,ebm->b", W, got)
    scale = np.einsum("em,ebm->b", W, np.abs(got))
    assert np.all(np.abs(tot) <= 1e-13 * scale), tot / scale


@pytest.fixture(scope="module")
def c2():
    return I.warped_workload()          # N = 7, 32768 elements, periodic 32^3 box


@pytest.mark.slow
def test_surface_full_n7_32768(sv, oracle_mod, c2):
    """The surface term at N = 7 on the whole periodic warped 32^3 box, FP64
    and FP32, in the launch the benchmark times."""
    ref = oracle_s(oracle_mod, c2)
    e = err(host(run(sv, c2)), ref)
    print("surface N=7 32768 fp64 err", e)
    assert e.max() <= TOL64
    ref32 = oracle_s(oracle_mod, c2, fp32=True)
    e32 = err(host(run(sv, c2, fp32=True)), ref32)
    print("surface N=7 32768 fp32 err", e32)
    assert e32.max() <= TOL32


# ---------------------------------------------------------------------------
# The whole rate v + s in one launch (sem_rhs)
# ---------------------------------------------------------------------------
def run_rhs(sv, w, nbr=None, with_ref=True, out=None, accumulate=False, fp32=False):
    src = I.to_fp32(w) if fp32 else w
    return sv.rhs(dev(src.q), dev(src.geo), dev(src.D), dev(w.nbr if nbr is None else nbr),
                  dev(src.rho_ref) if with_ref else None, dev(w.theta_ref) if with_ref else None,
                  w.phys.as_tuple(), out=out, accumulate=accumulate)


def oracle_vs(oracle_mod, w, nbr=None, with_ref=True, fp32=False):
    src = I.upcast(I.to_fp32(w)) if fp32 else w
    ph = w.phys.as_tuple()
    rr, tr = (src.rho_ref, w.theta_ref) if with_ref else (None, None)
    v = oracle_mod.volume_rhs(src.D, src.geo, src.q, rr, tr, ph)
    return v + oracle_mod.surface_rhs(src.geo, src.q, w.nbr if nbr is None else nbr, tr, ph)


@pytest.mark.parametrize("Nq", list(range(2, 11)))
def test_rhs_vs_oracle(sv, oracle_mod, Nq):
    """v + s in one launch against the oracle's volume term plus its surface
    term, every order, on a periodic warped box (several tiles and a ragged
    tail): FP64 and FP32, with and without the reference state, overwrite
    and accumulate."""
    w = I.warped_workload(N=Nq - 1, n_side=4 if Nq <= 4 else 3, k=330 + Nq)
    for with_ref in (True, False):
        ref = oracle_vs(oracle_mod, w, with_ref=with_ref)
        e = err(host(run_rhs(sv, w, with_ref=with_ref)), ref)
        assert e.max() <= TOL64, (Nq, with_ref, e)
        base = np.random.default_rng(Nq).standard_normal(w.q.shape)
        out = dev(base.copy())
        run_rhs(sv, w, with_ref=with_ref, out=out, accumulate=True)
        assert err(host(out), base + ref).max() <= TOL64, (Nq, with_ref)
        ref32 = oracle_vs(oracle_mod, w, with_ref=with_ref, fp32=True)
        e32 = err(host(run_rhs(sv, w, with_ref=with_ref, fp32=True)), ref32)
        assert e32.max() <= TOL32, (Nq, with_ref, e32)
        b32 = base.astype(np.float32)
        out32 = dev(b32.copy())
        run_rhs(sv, w, with_ref=with_ref, out=out32, accumulate=True, fp32=True)
        assert err(host(out32), b32.astype(np.float64) + ref32).max() <= TOL32, (Nq, with_ref)


def err_per_element(out, ref):
    """|out_b - ref_b| / max|ref_b| maximised within each element: [Ne, field],
    each element judged at its own scale."""
    d = np.abs(np.asarray(out, np.float64) - ref).max(axis=2)
    m = np.abs(ref).max(axis=2)
    return np.where(m > 0, d / np.where(m > 0, m, 1.0), 0.0)


EPS32 = 2.0 ** -23


def fp32_full_pressure_gate(w32, ref, surface):
    """Per element and field, the gate of the FP32 form without a reference
    state: the full pressure p = p0 (R Theta / p0)^gamma is rounded in FP32 to
    a few ulp (log, multiply, exp) and enters the momentum fluxes; the
    contractions pass its rounding on amplified by at most
    3 max_i sum_n |D_in| max|g| max(1/J) within the element, and the face
    term (v + s) by at most 3 (N (N + 1) / 2) max|g| max(1/J) more.  Gate for
    U1..U3: TOL32 + 4 eps32 max|p| amp / max|ref_b|; other fields TOL32."""
    x = w32.phys.R * np.asarray(w32.q[:, 4], np.float64) / w32.phys.p0
    p_max = (w32.phys.p0 * x ** w32.phys.gamma).max(axis=1)
    g = np.asarray(w32.geo, np.float64)
    D = np.asarray(w32.D, np.float64)
    Nq = D.shape[0]
    spread = np.abs(D).sum(axis=1).max() + (Nq - 1) * Nq / 2.0 * surface
    amp = 3 * spread * np.abs(g[:, :9]).max(axis=(1, 2)) * g[:, 9].max(axis=1)
    m = np.abs(ref).max(axis=2)
    gate = np.full(m.shape, TOL32)
    gate[:, 1:4] += 4 * EPS32 * (p_max * amp)[:, None] / np.where(m[:, 1:4] > 0, m[:, 1:4], 1.0)
    return gate


@pytest.mark.parametrize("Nq", [4, 8])
def test_pressure_over_decades_of_theta(sv, oracle_mod, Nq):
    """Theta_ref at a scale drawn per element over five decades (R Theta / p0
    from about 1e-3 to 6e2 at atmospheric constants, so the logarithm of the
    equation of state runs through binary exponents from -9 to +10) and
    Theta / Theta_ref from 0.5 to 2 at every node (log1p far from small
    arguments in FP32): the volume term and v + s against the oracle, each
    element judged at its own scale, FP64 and FP32, with and without the
    reference state."""
    w = I.warped_workload(N=Nq - 1, n_side=3, k=360 + Nq)
    rng = np.random.default_rng(3600 + Nq)
    scale = 10.0 ** rng.uniform(0.0, 5.0, size=(w.Ne, 1))
    w.theta_ref = scale * rng.uniform(0.8, 1.25, size=w.theta_ref.shape)
    w.q[:, 4] = w.theta_ref * rng.uniform(0.5, 2.0, size=w.theta_ref.shape)
    ph = w.phys.as_tuple()
    w32 = I.to_fp32(w)
    u = I.upcast(w32)
    for with_ref in (True, False):
        rr, tr = (w.rho_ref, w.theta_ref) if with_ref else (None, None)
        v = oracle_mod.volume_rhs(w.D, w.geo, w.q, rr, tr, ph)
        got = sv.volume_rhs(dev(w.q), dev(w.geo), dev(w.D), dev(rr), dev(tr), ph)
        e = err_per_element(host(got), v).max(axis=0)
        assert e.max() <= TOL64, ("volume", Nq, with_ref, e)
        vs = oracle_vs(oracle_mod, w, with_ref=with_ref)
        e = err_per_element(host(run_rhs(sv, w, with_ref=with_ref)), vs).max(axis=0)
        assert e.max() <= TOL64, ("v + s", Nq, with_ref, e)
        v32 = oracle_mod.volume_rhs(u.D, u.geo, u.q, u.rho_ref if with_ref else None,
                                    w.theta_ref if with_ref else None, ph)
        got32 = sv.volume_rhs(dev(w32.q), dev(w32.geo), dev(w32.D),
                              dev(w32.rho_ref) if with_ref else None,
                              dev(w.theta_ref) if with_ref else None, ph)
        e32 = err_per_element(host(got32), v32)
        gate = TOL32 if with_ref else fp32_full_pressure_gate(w32, v32, surface=False)
        assert np.all(e32 <= gate), ("volume fp32", Nq, with_ref, e32.max(axis=0))
        vs32 = oracle_vs(oracle_mod, w, with_ref=with_ref, fp32=True)
        e32 = err_per_element(host(run_rhs(sv, w, with_ref=with_ref, fp32=True)), vs32)
        gate = TOL32 if with_ref else fp32_full_pressure_gate(w32, vs32, surface=True)
        assert np.all(e32 <= gate), ("v + s fp32", Nq, with_ref, e32.max(axis=0))
        print("decades of Theta Nq", Nq, "ref", with_ref, "fp32 err", e32.max(axis=0))


@pytest.mark.parametrize("Nq", [3, 8])
def test_rhs_boundary_faces(sv, oracle_mod, Nq):
    """A sub-mesh of the box with boundary faces (neighbours outside it, and
    indices beyond Ne or below -1): those faces add nothing, as in the
    oracle; the kernel reads nothing through them."""
    w = I.warped_workload(N=Nq - 1, n_side=4, n_elements=37, k=340 + Nq)
    nbr = w.nbr.copy()
    nbr[3, 1] = w.Ne + 5
    nbr[7, 4] = 2 ** 31 - 1
    nbr[11, 2] = -7
    assert (nbr < 0).any()
    assert err(host(run_rhs(sv, w, nbr=nbr)), oracle_vs(oracle_mod, w, nbr=nbr)).max() <= TOL64
    ref32 = oracle_vs(oracle_mod, w, nbr=nbr, fp32=True)
    assert err(host(run_rhs(sv, w, nbr=nbr, fp32=True)), ref32).max() <= TOL32
    none = np.full_like(w.nbr, -1)
    got = host(run_rhs(sv, w, nbr=none))
    v = host(sv.volume_rhs(dev(w.q), dev(w.geo), dev(w.D), dev(w.rho_ref), dev(w.theta_ref),
                           w.phys.as_tuple()))
    assert err(got, v).max() <= TOL64


def test_rhs_conservative(sv, oracle_mod):
    """The GLL quadrature of J (v + s) over the periodic box vanishes (no
    gravity), for the one-launch rate as for the oracle's."""
    N = 4
    w = I.warped_workload(N=N, n_side=4, k=342)
    phys = (I.P0, I.GAMMA, I.R_GAS, 0.0)
    got = host(sv.rhs(dev(w.q), dev(w.geo), dev(w.D), dev(w.nbr), dev(w.rho_ref),
                      dev(w.theta_ref), phys))
    wq = I.gll_weights(N)
    Nq = N + 1
    m = np.arange(Nq ** 3)
    W = (wq[m % Nq] * wq[(m // Nq) % Nq] * wq[m // (Nq * Nq)])[None, :] / w.geo[:, 9]
    tot = np.einsum("em,ebm->b", W, got)
    scale = np.einsum("em,ebm->b", W, np.abs(got))
    assert np.all(np.abs(tot) <= 1e-13 * scale), tot / scale


@pytest.mark.slow
def test_rhs_full_n7_32768(sv, oracle_mod, c2):
    """v + s at N = 7 on the whole periodic warped 32^3 box, FP64 and FP32, in
    the launch the benchmark times."""
    ref = oracle_vs(oracle_mod, c2)
    e = err(host(run_rhs(sv, c2)), ref)
    print("rhs N=7 32768 fp64 err", e)
    assert e.max() <= TOL64
    ref32 = oracle_vs(oracle_mod, c2, fp32=True)
    e32 = err(host(run_rhs(sv, c2, fp32=True)), ref32)
    print("rhs N=7 32768 fp32 err", e32)
    assert e32.max() <= TOL32


def test_rhs_and_surface_inside_a_captured_graph(sv):
    """sem_rhs and sem_surface_rhs (accumulating) record into a captured HIP
    graph; every replay, with eager work between replays, equals the eager
    result bit for bit."""
    w = I.warped_workload(N=5, n_side=3, k=350)
    ph = w.phys.as_tuple()
    q, geo, D, nbr, rr, tr = (dev(a) for a in (w.q, w.geo, w.D, w.nbr, w.rho_ref, w.theta_ref))
    eager = sv.rhs(q, geo, D, nbr, rr, tr, ph)
    sv.surface_rhs(q, geo, nbr, tr, ph, out=eager, accumulate=True)
    out = torch.empty_like(q)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            sv.rhs(q, geo, D, nbr, rr, tr, ph, out=out)
            sv.surface_rhs(q, geo, nbr, tr, ph, out=out, accumulate=True)
    torch.cuda.current_stream().wait_stream(s)
    for replay in range(3):
        out.fill_(float("nan"))
        sv.volume_rhs(q, geo, D, rr, tr, ph)           # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), replay


def test_surface_and_rhs_deterministic(sv):
    """Two launches of the surface pass and of the whole rate give the same
    bits (each face node's flux is computed by one thread and every node sums
    its faces in a fixed order)."""
    w = I.warped_workload(N=7, n_side=4, k=360)
    ph = w.phys.as_tuple()
    q, geo, D, nbr, rr, tr = (dev(a) for a in (w.q, w.geo, w.D, w.nbr, w.rho_ref, w.theta_ref))
    for _ in range(2):
        a = host(sv.surface_rhs(q, geo, nbr, tr, ph))
        b = host(sv.surface_rhs(q, geo, nbr, tr, ph))
        assert np.array_equal(a, b)
        c = host(sv.rhs(q, geo, D, nbr, rr, tr, ph))
        d = host(sv.rhs(q, geo, D, nbr, rr, tr, ph))
        assert np.array_equal(c, d)
