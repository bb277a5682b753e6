"""The C-ABI library loads on the host and exports every entry point its header
declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "itokmc.h")
LIB = os.path.join(ROOT, "paper_2307_01797_amd", "libitokmc.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(itokmc_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("itokmc_init_grid", "itokmc_seed_particles", "itokmc_set_coefficients",
              "itokmc_step", "itokmc_deposit", "itokmc_diagnostics"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_export_list_matches_header():
    from paper_2307_01797_amd import itokmc
    assert sorted(itokmc.EXPORTS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_arena_size_and_descriptor_validation():
    from paper_2307_01797_amd import itokmc, workloads
    L = itokmc.lib()
    d = itokmc.make_desc(workloads.preset("avalanche_32"), max_particles=1000)
    n = L.itokmc_arena_bytes(ctypes.byref(d))
    assert n > 32**3 * 8
    bad = itokmc.make_desc(workloads.preset("avalanche_32"), max_particles=1000)
    bad.n_new = 65
    assert L.itokmc_arena_bytes(ctypes.byref(bad)) == 0
    bad = itokmc.make_desc(workloads.preset("avalanche_32", grid=(512, 512, 512)))
    assert L.itokmc_arena_bytes(ctypes.byref(bad)) == 0
    # init rejects a null arena without touching the device
    h = ctypes.c_void_p()
    assert L.itokmc_init_grid(ctypes.byref(h), ctypes.byref(d), None, n, None) == itokmc.EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_ensemble_descriptor_validation():
    from paper_2307_01797_amd import itokmc
    L = itokmc.lib()
    ok = itokmc.EnsDesc(256, itokmc.FP32, 1 << 26, 100_000_000)
    n = L.itokmc_ensemble_arena_bytes(ctypes.byref(ok))
    # two banks of 32 bytes per particle plus 36 bytes per pool cell, at least
    assert n >= 2 * 32 * 100_000_000 + 36 * (1 << 26)
    for bad in (itokmc.EnsDesc(0, itokmc.FP32, 4096, 1000),
                itokmc.EnsDesc(5000, itokmc.FP32, 4096, 1000),
                itokmc.EnsDesc(4, 7, 4096, 1000),
                itokmc.EnsDesc(4, itokmc.FP32, (1 << 31) + 1, 1000),
                itokmc.EnsDesc(4, itokmc.FP32, 4096, 1 << 31)):
        assert L.itokmc_ensemble_arena_bytes(ctypes.byref(bad)) == 0
    h = ctypes.c_void_p()
    assert L.itokmc_ensemble_create(ctypes.byref(h), ctypes.byref(ok), None, n, None) == itokmc.EINVAL
    assert L.itokmc_ensemble_step(None, 1) == itokmc.EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_coefficient_validation_on_host():
    import math

    from paper_2307_01797_amd import itokmc, workloads
    L = itokmc.lib()
    good = itokmc.make_coeffs(workloads.preset("streamer_64"))
    assert L.itokmc_check_coefficients(ctypes.byref(good)) == itokmc.OK
    for name, bad in (("D", math.nan), ("mu_a", math.inf), ("eta", -1.0), ("alpha_B", math.nan),
                      ("mu_E0", 0.0), ("E_floor", -5.0), ("photon_l1", math.nan)):
        c = itokmc.make_coeffs(workloads.preset("streamer_64"))
        setattr(c, name, bad)
        assert L.itokmc_check_coefficients(ctypes.byref(c)) == itokmc.EINVAL, name
    # photon lengths must be ordered when photons are emitted
    c = itokmc.make_coeffs(workloads.preset("streamer_64"))
    c.photon_l1, c.photon_l2 = 2e-3, 30e-6
    assert L.itokmc_check_coefficients(ctypes.byref(c)) == itokmc.EINVAL
    assert L.itokmc_check_coefficients(None) == itokmc.EINVAL
    assert L.itokmc_set_coefficients(None, ctypes.byref(good)) == itokmc.EINVAL


def test_binding_structs_match_header_layout(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets that the C
    compiler gives the header's struct (a field added on one side only fails here)."""
    import ctypes
    import shutil
    import subprocess

    from paper_2307_01797_amd import itokmc as b
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    pairs = {"itokmc_grid_desc": b.GridDesc, "itokmc_coeffs": b.Coeffs,
             "itokmc_seed_desc": b.SeedDesc, "itokmc_diag": b.Diag, "itokmc_tuning": b.Tuning,
             "itokmc_ens_desc": b.EnsDesc, "itokmc_run_desc": b.RunDesc,
             "itokmc_slot_event": b.SlotEvent, "itokmc_ens_info": b.EnsInfo,
             "itokmc_ens_tuning": b.EnsTuning, "itokmc_dt_rule": b.DtRule}
    lines = ['#include <stdio.h>', '#include "itokmc.h"', "int main(void) {"]
    for cname, cls in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, cls in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_oracle_binding_structs_match_header_layout(tmp_path):
    """The oracle's ctypes structures against its C header, as above."""
    import ctypes
    import shutil
    import subprocess

    import oracle as o
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    pairs = {"or_desc": o.Desc, "or_coeffs": o.Coeffs, "or_diag": o.Diag, "or_dt_rule": o.DtRule}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "oracle.h"', "int main(void) {"]
    for cname, cls in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "oracle"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, cls in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_library_rates_equal_oracle_rates_on_host():
    """itokmc_rates is host code: it runs without a GPU and equals the oracle's rates
    bit for bit (fields below, at and above the mobility floor; with and without
    recombination)."""
    import oracle

    from paper_2307_01797_amd import itokmc, workloads
    for coeffs in ({}, dict(workloads.RECOMBINATION), dict(kgamma_ratio=0.06)):
        cfg = workloads.preset("avalanche_32", coeffs=coeffs)
        for E in (0.0, 5e3, 1e4, 1.7e6, 1e7, 3.3e7):
            assert np.array_equal(itokmc.rates(cfg, E), oracle.rates(cfg, E)), (coeffs, E)
    with pytest.raises(itokmc.ItokmcError):
        itokmc.rates(workloads.preset("avalanche_32"), -1.0)


def test_binding_constants_match_header(tmp_path):
    """Every numeric constant of the binding (error codes, slot states, precisions,
    modes, shapes, query selectors, overflow flags) equals the header's enumerator."""
    import shutil
    import subprocess

    from paper_2307_01797_amd import itokmc as b
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    names = ["OK", "EINVAL", "ENOMEM", "ECAPACITY", "ENOCONV", "EHIP", "EAGAIN", "SLOT_FREE",
             "SLOT_ACTIVE", "SLOT_DONE", "SLOT_CAPPED", "FP32", "FP64", "FIELD_UNIFORM",
             "FIELD_POISSON", "KMC_HYBRID", "KMC_PURE_TAU", "SEED_GAUSSIAN", "SEED_NEUTRAL",
             "Q_NGP_WEIGHT", "Q_NPLUS", "Q_NMINUS", "Q_NGAMMA", "Q_CIC_DENSITY", "Q_PHI", "Q_EX",
             "Q_EY", "Q_EZ", "Q_FIRES", "Q_RHO", "OVF_PARTICLES", "OVF_MERGE", "OVF_BARRIER"]
    lines = ['#include <stdio.h>', '#include "itokmc.h"', "int main(void) {"]
    lines += [f'  printf("{n} %d\\n", (int)ITOKMC_{n});' for n in names]
    lines += ['  printf("SHAPE_CIC %d\\n", (int)ITOKMC_SHAPE_CIC);',
              '  printf("SHAPE_TSC %d\\n", (int)ITOKMC_SHAPE_TSC);', "  return 0;", "}"]
    src = tmp_path / "consts.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "consts"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict((k, int(v)) for k, v in (l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines()))
    for n in names:
        assert getattr(b, n) == got[n], n
    assert b.SHAPES == {"cic": got["SHAPE_CIC"], "tsc": got["SHAPE_TSC"]}
