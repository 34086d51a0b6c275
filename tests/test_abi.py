"""CPU checks of the C-ABI: libsem.so loads, exports every function that
include/sem.h declares, and rejects invalid arguments on the host before any
HIP call (every call below fails validation, so no kernel is launched and no
device memory is touched)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sem.h")


@pytest.fixture(scope="module")
def L():
    from paper_1604_08501_amd import semvol
    if not os.path.exists(semvol.LIB_PATH):
        from paper_1604_08501_amd import build
        build.build()
    return semvol.lib()


@pytest.fixture(scope="module")
def sv():
    from paper_1604_08501_amd import semvol
    return semvol


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sem_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L, sv):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(sv.EXPORTS)


def test_version(L):
    assert b"gfx950" in L.sem_version()


def test_tile_options(L, sv):
    buf = (sv.sem_tile * 16)()
    for nq in range(2, 11):
        n = L.sem_tile_options(sv.SEM_F64, nq, buf, 16)
        assert n >= 1
        assert all(buf[i].elems_per_block >= 1 for i in range(n))
        assert all(buf[i].layout in (sv.SEM_LAYOUT_FULL, sv.SEM_LAYOUT_ALIAS) for i in range(n))
        assert (buf[0].elems_per_block, buf[0].layout) != (0, 0)
    assert L.sem_tile_options(sv.SEM_F64, 11, buf, 16) == 0
    assert L.sem_tile_options(7, 8, buf, 16) == 0
    # large orders have an aliased-LDS shape
    assert ("alias" in [lay for _, lay in sv.tile_options(__import__("torch").float64, 10)])


# fake, suitably aligned device addresses: validation must fail before use
A = 0x10000


def _vol(L, sv, Ne=4, Nq=5, dt=0, D=A, geo=2 * A, q=3 * A, rr=None, tr=None, rhs=4 * A,
         phys=True, acc=0):
    ph = sv.sem_phys(1e5, 1.4, 287.0, 9.81)
    return L.sem_volume_rhs(Ne, Nq, dt, D, geo, q, rr, tr, ctypes.byref(ph) if phys else None,
                            rhs, acc, None)


@pytest.mark.parametrize("kw,status", [
    (dict(Ne=0), -1), (dict(Ne=-3), -1),
    (dict(Nq=1), -2), (dict(Nq=11), -2),
    (dict(dt=5), -1),
    (dict(D=None), -1), (dict(geo=None), -1), (dict(q=None), -1), (dict(rhs=None), -1),
    (dict(rr=5 * A), -1), (dict(tr=5 * A), -1),
    (dict(q=3 * A + 4), -1), (dict(dt=1, q=3 * A + 2), -1), (dict(rr=5 * A, tr=6 * A + 4), -1),
    (dict(rhs=3 * A), -1),
    (dict(phys=False), -1),
])
def test_volume_rhs_validation(L, sv, kw, status):
    assert _vol(L, sv, **kw) == status
    assert len(L.sem_last_error()) > 0


def test_tiled_rejects_uncompiled_shape(L, sv):
    ph = sv.sem_phys(1e5, 1.4, 287.0, 9.81)
    for tile, status in ((sv.sem_tile(3, 0), sv.SEM_ERR_UNSUPPORTED),
                         (sv.sem_tile(1, sv.SEM_LAYOUT_ALIAS), sv.SEM_ERR_UNSUPPORTED),  # Nq = 4
                         (sv.sem_tile(1, 9), sv.SEM_ERR_INVALID_ARG)):
        st = L.sem_volume_rhs_tiled(4, 4, 0, A, 2 * A, 3 * A, None, None, ctypes.byref(ph), 4 * A, 0,
                                    ctypes.byref(tile), None)
        assert st == status
        assert b"tile" in L.sem_last_error() or b"layout" in L.sem_last_error()


def test_adjoint_validation(L, sv):
    ph = sv.sem_phys(1e5, 1.4, 287.0, 9.81)
    assert L.sem_volume_rhs_adjoint(0, 8, 0, A, 2 * A, 3 * A, ctypes.byref(ph), 4 * A, 5 * A, 0,
                                    None) == -1
    assert L.sem_volume_rhs_adjoint(4, 8, 0, A, 2 * A, 3 * A, ctypes.byref(ph), None, 5 * A, 0,
                                    None) == -1
    assert L.sem_volume_rhs_adjoint(4, 8, 0, A, 2 * A, 3 * A, ctypes.byref(ph), 4 * A, 4 * A, 0,
                                    None) == -1
    assert L.sem_volume_rhs_adjoint(4, 12, 0, A, 2 * A, 3 * A, ctypes.byref(ph), 4 * A, 5 * A, 0,
                                    None) == -2


def test_axpby_validation(L, sv):
    assert L.sem_axpby(-1, 0, 1.0, A, 1.0, A, 1.0, A, A, None) == -1
    assert L.sem_axpby(10, 0, 1.0, None, 1.0, A, 1.0, A, A, None) == -1   # x needed when a != 0
    assert L.sem_axpby(10, 3, 1.0, A, 1.0, A, 1.0, A, A, None) == -1
    assert L.sem_axpby(10, 0, 0.0, None, 1.0, A + 1, 1.0, A, A, None) == -1


def test_batch_plan_validation(L, sv):
    ph = sv.sem_phys(1e5, 1.4, 287.0, 9.81)
    out = ctypes.c_void_p()
    blocks = (sv.sem_block * 2)()
    blocks[0] = sv.sem_block(5, 10, A, 2 * A, 3 * A, None, None, 4 * A)
    blocks[1] = sv.sem_block(13, 10, A, 2 * A, 3 * A, None, None, 4 * A)     # Nq not compiled
    assert L.sem_batch_plan(blocks, 0, 0, ctypes.byref(ph), 0, None, ctypes.byref(out)) == -1
    assert L.sem_batch_plan(blocks, 2, 0, ctypes.byref(ph), 0, None, ctypes.byref(out)) == -2
    assert b"block 1" in L.sem_last_error()
    assert not out.value
    assert L.sem_batch_execute(None, None) == -1
    assert L.sem_plan_destroy(None) == -1
    buf = ctypes.create_string_buffer(16)
    assert L.sem_plan_describe(None, buf, 16) == -1


def test_batch_rhs_static_validation(L, sv):
    """The entry point without allocation rejects, on the host, what the plan
    rejects and what exceeds its static tables (more than 16 blocks, more
    than 32768 tiles)."""
    ph = sv.sem_phys(1e5, 1.4, 287.0, 9.81)
    blocks = (sv.sem_block * 17)()
    for i in range(17):
        base = (i + 1) << 40
        blocks[i] = sv.sem_block(5, 10, base, base + (1 << 36), base + (2 << 36), None, None,
                                 base + (3 << 36))
    assert L.sem_batch_rhs_static(blocks, 0, 0, ctypes.byref(ph), None) == -1
    assert L.sem_batch_rhs_static(blocks, 17, 0, ctypes.byref(ph), None) == -1
    assert b"16 blocks" in L.sem_last_error()
    assert L.sem_batch_rhs_static(blocks, 2, 0, None, None) == -1
    assert L.sem_batch_rhs_static(blocks, 2, 5, ctypes.byref(ph), None) == -1
    blocks[1] = sv.sem_block(13, 10, A, 2 * A, 3 * A, None, None, 4 * A)     # Nq not compiled
    assert L.sem_batch_rhs_static(blocks, 2, 0, ctypes.byref(ph), None) == -2
    assert b"block 1" in L.sem_last_error()
    # 40000 elements at Nq = 10 are 40000 one-element tiles
    b = 1 << 44
    big = (sv.sem_block * 1)(sv.sem_block(10, 40000, b, b + (1 << 40), b + (2 << 40), None, None,
                                          b + (3 << 40)))
    assert L.sem_batch_rhs_static(big, 1, 0, ctypes.byref(ph), None) == -1
    assert b"static tile table" in L.sem_last_error()
    # rhs overlapping q
    bad = (sv.sem_block * 1)(sv.sem_block(5, 10, A, 2 * A, 3 * A, None, None, 3 * A + 16))
    assert L.sem_batch_rhs_static(bad, 1, 0, ctypes.byref(ph), None) == -1


def test_binding_rejects_an_empty_block_list(sv):
    with pytest.raises(ValueError, match="at least one block"):
        sv.batch_rhs_static([])
    with pytest.raises(ValueError, match="at least one block"):
        sv.BatchPlan([])


def test_rk3_validation(L, sv):
    ph = sv.sem_phys(1e5, 1.4, 287.0, 9.81)
    out = ctypes.c_void_p()
    blocks = (sv.sem_block * 1)()
    M = 5 ** 3
    blocks[0] = sv.sem_block(5, 2, A, 2 * A, 3 * A, None, None, 4 * A)
    # q not inside q_n
    assert L.sem_rk3_graph_create(blocks, 1, 0, ctypes.byref(ph), 0, 8 * A, 9 * A, 10 * A, 4 * A,
                                  2 * 5 * M, 1e-3, None, ctypes.byref(out)) == -1
    # rhs not at the same offset in L as q in q_n
    assert L.sem_rk3_graph_create(blocks, 1, 0, ctypes.byref(ph), 0, 3 * A, 9 * A, 10 * A,
                                  4 * A - 8, 2 * 5 * M, 1e-3, None, ctypes.byref(out)) == -1
    assert L.sem_rk3_graph_create(blocks, 1, 0, ctypes.byref(ph), 0, 3 * A, 9 * A, 10 * A, 4 * A,
                                  0, 1e-3, None, ctypes.byref(out)) == -1
    assert L.sem_rk3_graph_launch(None, None) == -1
    assert L.sem_rk3_graph_destroy(None) == -1
    buf = ctypes.create_string_buffer(16)
    assert L.sem_rk3_graph_describe(None, buf, 16) == -1


def test_binding_fails_loudly_without_library(monkeypatch):
    from paper_1604_08501_amd import semvol
    monkeypatch.setattr(semvol, "_lib", None)
    monkeypatch.setattr(semvol, "LIB_PATH", "/nonexistent/libsem.so")
    with pytest.raises(ImportError):
        semvol.lib()


def test_ext_validation(L, sv):
    ph = sv.sem_phys(1.0, 1.4, 1.0, 0.0)

    def ext(Ne=4, Nq=8, dt=1, nf=8, dirs=3, q=3 * A, rhs=4 * A):
        return L.sem_volume_rhs_ext(Ne, Nq, dt, nf, dirs, A, 2 * A, q, None, None,
                                    ctypes.byref(ph), rhs, 0, None)
    assert ext(Ne=0) == sv.SEM_ERR_INVALID_ARG
    assert ext(nf=6) == sv.SEM_ERR_UNSUPPORTED
    assert ext(dirs=5) == sv.SEM_ERR_UNSUPPORTED
    assert ext(dirs=1) == sv.SEM_ERR_UNSUPPORTED
    assert ext(Nq=11) == sv.SEM_ERR_UNSUPPORTED
    assert b"Nq = 11" in L.sem_last_error()
    assert ext(q=3 * A + 2) == sv.SEM_ERR_INVALID_ARG      # misaligned FP32 array
    assert ext(rhs=3 * A) == sv.SEM_ERR_INVALID_ARG        # rhs aliases q
    assert ext(dt=9) == sv.SEM_ERR_INVALID_ARG


def test_affine_validation(L, sv):
    ph = sv.sem_phys(1e5, 1.4, 287.0, 9.81)

    def aff(Ne=4, Nq=8, dt=0, geo=2 * A, rhs=4 * A):
        return L.sem_volume_rhs_affine(Ne, Nq, dt, A, geo, 3 * A, None, None, ctypes.byref(ph),
                                       rhs, 0, None)
    assert aff(Ne=0) == sv.SEM_ERR_INVALID_ARG
    assert aff(Nq=11) == sv.SEM_ERR_UNSUPPORTED
    assert aff(geo=None) == sv.SEM_ERR_INVALID_ARG
    assert aff(geo=2 * A + 4) == sv.SEM_ERR_INVALID_ARG
    assert aff(rhs=2 * A) == sv.SEM_ERR_INVALID_ARG


def test_ladder_validation(L, sv):
    ph = sv.sem_phys(1.0, 1.4, 1.0, 0.0)
    grav = sv.sem_phys(1.0, 1.4, 1.0, 9.81)

    def lad(level=1, Ne=4, Nq=8, q=3 * A, rhs=4 * A, phys=ph):
        return L.sem_volume_rhs_ladder(level, Ne, Nq, A, 2 * A, q, ctypes.byref(phys), rhs, None)
    assert lad(level=0) == sv.SEM_ERR_INVALID_ARG
    assert lad(level=7) == sv.SEM_ERR_INVALID_ARG
    assert b"level" in L.sem_last_error()
    assert lad(Ne=0) == sv.SEM_ERR_INVALID_ARG
    assert lad(Nq=11) == sv.SEM_ERR_UNSUPPORTED
    assert lad(Nq=1) == sv.SEM_ERR_UNSUPPORTED
    assert lad(phys=grav) == sv.SEM_ERR_UNSUPPORTED
    assert lad(q=3 * A + 2) == sv.SEM_ERR_INVALID_ARG
    assert lad(rhs=3 * A) == sv.SEM_ERR_INVALID_ARG
    assert L.sem_volume_rhs_ladder(1, 4, 8, A, 2 * A, 3 * A, None, 4 * A, None) == \
        sv.SEM_ERR_INVALID_ARG


def test_last_error_is_per_thread(L, sv):
    """Each thread reads the message of its own last failure."""
    import threading
    ph = sv.sem_phys(1e5, 1.4, 287.0, 9.81)
    A = 1 << 20
    seen = {}
    barrier = threading.Barrier(2)

    def worker(name, Ne, Nq):
        st = L.sem_volume_rhs(Ne, Nq, 0, A, 2 * A, 3 * A, None, None, ctypes.byref(ph), 4 * A, 0,
                              None)
        barrier.wait()          # both threads have failed before either reads
        seen[name] = (st, L.sem_last_error().decode())

    t1 = threading.Thread(target=worker, args=("a", 0, 8))
    t2 = threading.Thread(target=worker, args=("b", 4, 11))
    t1.start(); t2.start(); t1.join(); t2.join()
    assert seen["a"][0] == sv.SEM_ERR_INVALID_ARG and "Ne = 0" in seen["a"][1]
    assert seen["b"][0] == sv.SEM_ERR_UNSUPPORTED and "Nq = 11" in seen["b"][1]


C_CLIENT = r"""
#include <stdio.h>
#include <string.h>
#include "sem.h"
int main(void)
{
    sem_phys ph = {1e5, 1.4, 287.0, 9.81};
    sem_tile tiles[64];
    int n = sem_tile_options(SEM_F64, 8, tiles, 64);
    sem_status st = sem_volume_rhs(0, 8, SEM_F64, (void*)0x10000, (void*)0x20000, (void*)0x30000,
                                   NULL, NULL, &ph, (void*)0x40000, 0, NULL);
    printf("%s|%d|%d|%s\n", sem_version(), n, (int)st, sem_last_error());
    return (n > 0 && st == SEM_ERR_INVALID_ARG) ? 0 : 1;
}
"""


def test_c_client_compiles_links_and_calls(L, tmp_path):
    """include/sem.h compiles as C99 (and C++11) and a C program linked
    against libsem.so calls through it (host-side validation only)."""
    import shutil
    import subprocess
    from paper_1604_08501_amd import semvol
    if not shutil.which("gcc") or not shutil.which("g++"):
        pytest.skip("no host C compiler")
    src = tmp_path / "client.c"
    src.write_text(C_CLIENT)
    inc = os.path.join(ROOT, "include")
    libdir = os.path.dirname(semvol.LIB_PATH)
    exe = tmp_path / "client"
    subprocess.run(["g++", "-std=c++11", "-Wall", "-Wextra", "-pedantic", "-fsyntax-only", "-x",
                    "c++", f"-I{inc}", str(src)], check=True)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", f"-I{inc}", str(src),
                    f"-L{libdir}", "-l:libsem.so", f"-Wl,-rpath,{libdir}", "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    version, n, status, msg = r.stdout.strip().split("|", 3)
    assert version.startswith("semvol") and int(n) > 0
    assert int(status) == -1 and "Ne = 0" in msg


# ---------------------------------------------------------------------------
# Overlapping outputs, the RK3 block tiling and the workgroup cap
# ---------------------------------------------------------------------------
B = 1 << 24          # far apart: the arrays below never overlap unless placed to


def test_rhs_partially_overlapping_an_input_is_rejected(L, sv):
    """rhs is written while q, geo, D and the reference are read: any shared
    byte, not only an equal pointer, is rejected before a launch."""
    ph = sv.sem_phys(1e5, 1.4, 287.0, 9.81)
    Ne, Nq = 4, 5
    M = Nq ** 3
    q, geo, D, rr, tr = B, 2 * B, 3 * B, 4 * B, 5 * B
    qbytes = Ne * 5 * M * 8

    def vol(rhs):
        return L.sem_volume_rhs(Ne, Nq, 0, D, geo, q, rr, tr, ctypes.byref(ph), rhs, 0, None)
    # last value of rhs on the first value of q; rhs starting inside q, geo,
    # D, rho_ref, theta_ref
    for rhs in (q - qbytes + 8, q + 8, geo + 10 * M * 8, D + 8, rr + 16, tr + Ne * M * 8 - 8):
        assert vol(rhs) == sv.SEM_ERR_INVALID_ARG, hex(rhs)
        assert b"overlaps" in L.sem_last_error()
    # touching but disjoint ranges are fine: validation passes, so the call
    # would launch; check only that the overlap check is not what fails by
    # asking for an unsupported order with the same pointers
    assert L.sem_volume_rhs(Ne, 11, 0, D, geo, q, rr, tr, ctypes.byref(ph), q + qbytes, 0,
                            None) == sv.SEM_ERR_UNSUPPORTED
    assert sv.lib().sem_volume_rhs_affine(Ne, Nq, 0, D, geo, q, rr, tr, ctypes.byref(ph),
                                          geo + 8 * 8, 0, None) == sv.SEM_ERR_INVALID_ARG
    ext = lambda rhs, nf: L.sem_volume_rhs_ext(Ne, 8, 1, nf, 3, D, geo, q, None, None,
                                                ctypes.byref(ph), rhs, 0, None)
    # with 8 fields the q array is 8/5 as long: rhs just past the 5-field
    # extent still overlaps it
    assert ext(q + Ne * 5 * 512 * 4, 8) == sv.SEM_ERR_INVALID_ARG


def test_adjoint_mu_partial_overlap(L, sv):
    ph = sv.sem_phys(1e5, 1.4, 287.0, 9.81)
    Ne, Nq = 3, 4
    lam = 4 * B
    assert L.sem_volume_rhs_adjoint(Ne, Nq, 0, B, 2 * B, 3 * B, ctypes.byref(ph), lam,
                                    lam + 64, 0, None) == sv.SEM_ERR_INVALID_ARG
    assert b"overlaps lambda" in L.sem_last_error()


def test_axpby_overlap_rules(L, sv):
    n = 1000
    # out shifted by one value against y: a race, rejected
    assert L.sem_axpby(n, 0, 1.0, B, 1.0, 2 * B, 1.0, 3 * B, 2 * B + 8, None) == \
        sv.SEM_ERR_INVALID_ARG
    assert b"overlaps y" in L.sem_last_error()
    assert L.sem_axpby(n, 0, 1.0, B, 1.0, 2 * B, 1.0, 3 * B, 3 * B - 8, None) == \
        sv.SEM_ERR_INVALID_ARG
    # x is not read when a == 0, so an overlap with it does not matter: the
    # call then fails only on the unknown dtype
    assert L.sem_axpby(n, 7, 0.0, 2 * B + 8, 1.0, 2 * B, 1.0, 3 * B, 4 * B, None) == \
        sv.SEM_ERR_INVALID_ARG
    assert b"dtype" in L.sem_last_error()


def _rk3(L, sv, blocks, q_n, L_buf, n, q1=20 * B, q2=30 * B):
    ph = sv.sem_phys(1e5, 1.4, 287.0, 9.81)
    out = ctypes.c_void_p()
    arr = (sv.sem_block * len(blocks))(*blocks)
    st = L.sem_rk3_graph_create(arr, len(blocks), 0, ctypes.byref(ph), 0, q_n, q1, q2, L_buf, n,
                                1e-3, None, ctypes.byref(out))
    assert not out.value
    return st


def test_rk3_blocks_must_tile_q_n(L, sv):
    """A gap between the blocks (values of q_n no stage would advance in the
    fused mode, and would mix with unset L values in the separate mode), an
    overlap, or a tail left over are rejected before anything is enqueued."""
    Nq, Ne = 4, 3
    sz = Ne * 5 * Nq ** 3 * 8          # bytes of one block's q
    qn, Lb = 2 * B, 8 * B

    def blk(off):
        return sv.sem_block(Nq, Ne, B, 40 * B, qn + off, None, None, Lb + off)
    n = 2 * sz // 8
    assert _rk3(L, sv, [blk(0), blk(sz + 8)], qn, Lb, n + 1) == sv.SEM_ERR_INVALID_ARG
    assert b"gap" in L.sem_last_error()
    assert _rk3(L, sv, [blk(0), blk(sz - 8)], qn, Lb, n) == sv.SEM_ERR_INVALID_ARG
    assert b"overlap" in L.sem_last_error()
    assert _rk3(L, sv, [blk(0), blk(sz)], qn, Lb, n + 5) == sv.SEM_ERR_INVALID_ARG
    assert b"cover" in L.sem_last_error()
    # q_1 overlapping q_n
    assert _rk3(L, sv, [blk(0), blk(sz)], qn, Lb, n, q1=qn + 8) == sv.SEM_ERR_INVALID_ARG
    assert b"overlaps" in L.sem_last_error()


def test_max_workgroups_setter(L, sv):
    assert L.sem_set_max_workgroups(-1) == sv.SEM_ERR_INVALID_ARG
    assert L.sem_set_max_workgroups(7) == sv.SEM_OK
    assert L.sem_set_max_workgroups(0) == sv.SEM_OK


def test_surface_validation(L, sv):
    ph = sv.sem_phys(1e5, 1.4, 287.0, 9.81)
    Ne, Nq = 4, 5
    M = Nq ** 3

    def surf(Ne=Ne, Nq=Nq, dt=0, nbr=B, geo=2 * B, q=3 * B, tr=None, rhs=4 * B, phys=True):
        return L.sem_surface_rhs(Ne, Nq, dt, nbr, geo, q, tr, ctypes.byref(ph) if phys else None,
                                 rhs, 0, None)
    assert surf(Ne=0) == sv.SEM_ERR_INVALID_ARG
    assert surf(Nq=11) == sv.SEM_ERR_UNSUPPORTED
    assert surf(Nq=1) == sv.SEM_ERR_UNSUPPORTED
    assert surf(dt=4) == sv.SEM_ERR_INVALID_ARG
    assert surf(nbr=None) == sv.SEM_ERR_INVALID_ARG
    assert surf(nbr=B + 2) == sv.SEM_ERR_INVALID_ARG          # int32 table misaligned
    assert surf(q=3 * B + 4) == sv.SEM_ERR_INVALID_ARG
    assert surf(tr=5 * B + 4) == sv.SEM_ERR_INVALID_ARG
    assert surf(phys=False) == sv.SEM_ERR_INVALID_ARG
    assert surf(rhs=3 * B + 8) == sv.SEM_ERR_INVALID_ARG       # overlaps q
    assert b"overlaps q" in L.sem_last_error()
    assert surf(rhs=B + 16) == sv.SEM_ERR_INVALID_ARG          # overlaps the neighbour table
    assert b"overlaps nbr" in L.sem_last_error()
    assert surf(tr=5 * B, rhs=5 * B + Ne * M * 8 - 8) == sv.SEM_ERR_INVALID_ARG


def test_rhs_validation(L, sv):
    """The one-launch v + s rejects what the volume term and the surface
    term reject, before any HIP call."""
    ph = sv.sem_phys(1e5, 1.4, 287.0, 9.81)
    Ne, Nq = 4, 5
    M = Nq ** 3

    def rhs(Ne=Ne, Nq=Nq, dt=0, D=B, geo=2 * B, q=3 * B, rr=None, tr=None, nbr=5 * B, out=6 * B,
            phys=True):
        return L.sem_rhs(Ne, Nq, dt, D, geo, q, rr, tr, nbr, ctypes.byref(ph) if phys else None,
                         out, 0, None)
    assert rhs(Ne=0) == sv.SEM_ERR_INVALID_ARG
    assert rhs(Nq=12) == sv.SEM_ERR_UNSUPPORTED
    assert rhs(Nq=1) == sv.SEM_ERR_UNSUPPORTED
    assert rhs(dt=4) == sv.SEM_ERR_INVALID_ARG
    assert rhs(nbr=None) == sv.SEM_ERR_INVALID_ARG
    assert rhs(nbr=5 * B + 2) == sv.SEM_ERR_INVALID_ARG          # int32 table misaligned
    assert rhs(q=None) == sv.SEM_ERR_INVALID_ARG
    assert rhs(rr=4 * B) == sv.SEM_ERR_INVALID_ARG               # reference pair incomplete
    assert rhs(phys=False) == sv.SEM_ERR_INVALID_ARG
    assert rhs(out=3 * B + 8) == sv.SEM_ERR_INVALID_ARG          # overlaps q
    assert rhs(out=5 * B + 16) == sv.SEM_ERR_INVALID_ARG         # overlaps the neighbour table
    assert b"overlaps nbr" in L.sem_last_error()
