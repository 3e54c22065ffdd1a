"""The C ABI on its own: a plain C99 program (c_abi_driver.c), built with gcc
against include/rfa.h and librfa.so, with no Python, ctypes or torch in the
process, steps a seeded case (outputs held to the same parity rules against
the FP64 oracle as the binding's), batches copies of it (bitwise equal to a
copy stepped alone) and differentiates it (gradients bitwise those of the
binding on the same case)."""
from __future__ import annotations

import math
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import parity
from oracle import oracle as O
from paper_1907_05709_amd import rfa
from paper_1907_05709_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.dirname(rfa.LIB_PATH)


def _build(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not found")
    if not os.path.exists(rfa.LIB_PATH):
        pytest.fail("librfa.so not built (python -m paper_1907_05709_amd.build)")
    exe = str(tmp_path / "c_abi_driver")
    subprocess.run([cc, "-std=c99", "-O1", "-Wall", "-Werror",
                    os.path.join(ROOT, "tests", "c_abi_driver.c"), "-o", exe,
                    f"-L{LIBDIR}", "-lrfa", f"-Wl,-rpath,{LIBDIR}"], check=True)
    return exe


def _write_case(path, case):
    nx, ny, nz = case.shape
    b = bytearray()
    b += struct.pack("<3i3d", nx, ny, nz, *case.spacing)
    b += struct.pack("<5d", case.t_death, case.arrhenius_a, case.arrhenius_ea, case.gas_r,
                     case.omega_cap)
    b += struct.pack("<i", len(case.tissue))
    for t in case.tissue:
        b += struct.pack("<6d2i", t.k, t.rho, t.c, t.h, t.q_met, t.t_fixed, t.fixed, t.tissue)
    b += np.ascontiguousarray(case.labels, dtype=np.uint8).tobytes()
    nd = case.needle
    b += struct.pack("<i", len(nd.power))
    b += np.ascontiguousarray(nd.pt_offset, dtype="<i4").tobytes()
    b += np.ascontiguousarray(nd.pts, dtype="<f8").tobytes()
    b += np.ascontiguousarray(nd.power, dtype="<f8").tobytes()
    b += struct.pack("<ddi", nd.sigma, case.dt, case.n_steps)
    with open(path, "wb") as fh:
        fh.write(bytes(b))


def _read_out(path, shape):
    n = int(np.prod(shape))
    raw = open(path, "rb").read()
    assert len(raw) == 8 * n + n + 4 * n + 32
    T = np.frombuffer(raw, "<f8", n, 0).reshape(shape)
    mask = np.frombuffer(raw, np.uint8, n, 8 * n).reshape(shape)
    om = np.frombuffer(raw, "<f4", n, 9 * n).reshape(shape)
    energy, injected, residual = struct.unpack_from("<3d", raw, 13 * n)
    (mono,) = struct.unpack_from("<q", raw, 13 * n + 24)
    return T, mask, om, dict(energy_J=energy, injected_J=injected, residual_J=residual,
                             mono_violations=mono)


def test_header_case_file_round_trip_on_host(tmp_path):
    """Host part: the case file holds every field the driver reads, in order
    (checked by length against the format in c_abi_driver.c)."""
    case = W.random_tissue_case(41, shape=(9, 7, 5), n_classes=4, n_tines=2, n_steps=3)
    p = tmp_path / "case.bin"
    _write_case(p, case)
    n = int(np.prod(case.shape))
    nt = len(case.needle.power)
    npts = int(case.needle.pt_offset[-1])
    want = (12 + 24 + 40 + 4 + len(case.tissue) * 56 + n + 4 + 4 * (nt + 1) + 24 * npts + 8 * nt
            + 8 + 8 + 4)
    assert os.path.getsize(p) == want


@pytest.mark.gpu
@pytest.mark.parametrize("seed,shape", [(42, (29, 37, 70)), (43, (64, 9, 33))])
def test_c_program_matches_oracle(seed, shape, tmp_path):
    O.build(force=False)
    exe = _build(tmp_path)
    case = W.random_tissue_case(seed, shape=shape, n_classes=5, n_tines=3, n_steps=120)
    _write_case(tmp_path / "case.bin", case)
    print(f"c driver case seed {seed} shape {shape}", flush=True)
    r = subprocess.run([exe, str(tmp_path / "case.bin"), str(tmp_path / "out.bin")],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    print(r.stdout.strip())
    T, mask, om, d = _read_out(tmp_path / "out.bin", case.shape)
    ost, dg, _ = O.run(case, diag=True)
    err = parity.compare(case, T, mask, om, ost)
    print(f"c driver: max|dT| = {err:.3e} K")
    assert math.isclose(d["injected_J"], dg[:, 1].sum(), rel_tol=1e-9)
    assert math.isclose(d["energy_J"], dg[-1, 0], rel_tol=2e-5)
    scale = abs(dg[:, 1].sum()) + abs(dg[:, 2].sum()) + abs(dg[:, 3].sum())
    assert abs(d["residual_J"]) <= 1e-6 * scale


@pytest.mark.gpu
def test_c_program_batches_grids(tmp_path):
    """rfa_batch_create / rfa_batch_step / rfa_batch_get_plan /
    rfa_batch_destroy from C: two copies of a case stepped in one batch end
    bitwise equal to a third stepped alone."""
    exe = _build(tmp_path)
    case = W.random_tissue_case(45, shape=(30, 22, 41), n_classes=4, n_tines=2, n_steps=37)
    _write_case(tmp_path / "case.bin", case)
    r = subprocess.run([exe, str(tmp_path / "case.bin"), str(tmp_path / "out.bin"), "batch"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    print(r.stdout.strip())
    equal, layout, tile_y, tile_x, items, workgroups, groups = struct.unpack(
        "<7i", open(tmp_path / "out.bin", "rb").read())
    assert equal == 1
    assert layout in (rfa.RFA_BATCH_TILES, rfa.RFA_BATCH_FLAT) and items > 0 and groups >= 1


@pytest.mark.gpu
def test_c_program_adjoint_equals_binding(tmp_path):
    """rfa_set_perfusion_bspline / rfa_forward_checkpointed / rfa_adjoint
    from C give the binding's gradients bit for bit on the same case."""
    exe = _build(tmp_path)
    case = W.random_tissue_case(46, shape=(20, 18, 24), n_classes=4, n_tines=3, n_steps=40)
    _write_case(tmp_path / "case.bin", case)
    r = subprocess.run([exe, str(tmp_path / "case.bin"), str(tmp_path / "out.bin"), "adjoint"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    print(r.stdout.strip())
    nt = len(case.needle.power)
    raw = open(tmp_path / "out.bin", "rb").read()
    assert len(raw) == 8 * (nt + 64)
    dP_c = np.frombuffer(raw, "<f8", nt, 0)
    dc_c = np.frombuffer(raw, "<f8", 64, 8 * nt).reshape(4, 4, 4)
    g = rfa.Grid(case.shape, case.spacing, t_death=case.t_death, A=case.arrhenius_a,
                 Ea=case.arrhenius_ea, R=case.gas_r, omega_cap=case.omega_cap)
    g.load_case(case)
    g.set_perfusion_bspline(np.zeros((4, 4, 4), np.float32))
    g.forward_checkpointed(case.n_steps, case.dt, case.n_steps // 3 + 1)
    dP, dc, _ = g.adjoint(np.ones(case.shape, np.float32), nt, 4)
    g.close()
    assert np.abs(dP).max() > 0
    assert np.array_equal(dP, dP_c) and np.array_equal(dc, dc_c)


@pytest.mark.gpu
def test_c_program_reports_errors(tmp_path):
    """A dt above the stability bound comes back as RFA_ERR_UNSTABLE with
    its message on stderr and a non-zero exit, through the C ABI alone."""
    exe = _build(tmp_path)
    case = W.random_tissue_case(44, shape=(12, 10, 8), n_classes=3, n_tines=1, n_steps=2)
    case.dt = 1e3
    _write_case(tmp_path / "case.bin", case)
    r = subprocess.run([exe, str(tmp_path / "case.bin"), str(tmp_path / "out.bin")],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 1
    assert "rfa_step" in r.stderr and "stab" in r.stderr
    assert not os.path.exists(tmp_path / "out.bin")
