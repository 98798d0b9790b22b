"""The C-ABI library on the host: it loads, exports every declared entry point,
validates queries and plans boxes without a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2508_06012_amd import mdeos as m
from paper_2508_06012_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mdeos.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mdeos_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L = m.lib()
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(m.EXPORTED)


def test_version_and_strerror():
    assert "gfx950" in m.mdeos_version()
    assert m.lib().mdeos_strerror(m.INVALID_ARG) == b"invalid argument"


def spec(**kw):
    d = dict(rho=0.8442, e=1.07, n_c=4, rc=2.5, dt=0.005, seed=1, cell_id=0)
    d.update(kw)
    return m.make_specs(d["rho"], d["e"], d["n_c"], d["rc"], d["dt"], d["seed"], d["cell_id"])[0]


@pytest.mark.parametrize("bad", [dict(rho=0.0), dict(rho=-1.0), dict(e=0.0), dict(e=float("nan")), dict(n_c=0),
                                 dict(n_c=11), dict(rc=0.0), dict(dt=0.0), dict(rc=7.0)])
def test_invalid_specs_rejected(bad):
    assert m.mdeos_validate(spec(**bad)) == m.INVALID_ARG


@pytest.mark.parametrize("kw", [dict(n_steps=0, n_avg=1), dict(n_steps=100, n_avg=101), dict(n_steps=100, n_avg=50,
                                n_blocks=7), dict(n_steps=100, n_avg=50, rescale_steps=(51,)),
                                dict(n_steps=100, n_avg=50, energy_every=0), dict(n_steps=100, n_avg=50, n_blocks=1)])
def test_invalid_schedules_rejected(kw):
    d = dict(n_steps=100, n_avg=50, rescale_steps=(), n_blocks=10, energy_every=10)
    d.update(kw)
    s = m.make_schedule(d["n_steps"], d["n_avg"], d["rescale_steps"], d["n_blocks"], d["energy_every"])
    assert m.mdeos_validate(spec(), s) == m.INVALID_ARG


def test_valid_workload_cells_plan():
    for w in (wl.cfg1(), wl.cfg2(mesh=16)):
        specs, sch = m.specs_from_workload(w)
        for i in range(len(specs)):
            assert m.mdeos_validate(specs[i], sch) == m.OK
            p = m.mdeos_plan(specs[i])
            assert p.N == 4 * specs[i].n_c ** 3
            assert p.L == pytest.approx(specs[i].n_c * (4 / specs[i].rho) ** (1 / 3), rel=1e-6)
            assert p.rl > specs[i].rc and p.rl < p.L
            assert p.lds_bytes <= 160 * 1024
            assert p.list_cap % 8 == 0
            # the extended box holds the real atoms plus their periodic images
            assert p.ext_cap >= p.N


def test_default_skin_per_box_size():
    """skin <= 0 plans with the per-size LJTS default: 0.3 up to 150 atoms, 0.4
    up to 600 atoms or for rc > 3.5, 0.6 above."""
    cases = [(3, 0.8, 2.5, 0.3), (4, 0.8, 2.5, 0.4), (5, 0.8, 2.5, 0.4), (6, 0.8, 2.5, 0.6), (7, 0.8, 3.0, 0.6),
             (10, 0.8, 2.5, 0.6), (6, 0.8, 4.0, 0.4)]
    for n_c, rho, rc, skin in cases:
        s = spec(rho=rho, n_c=n_c, rc=rc)
        p = m.mdeos_plan(s, 0.0)
        assert p.rl == pytest.approx(rc + skin, abs=1e-6), (n_c, rho, rc, p.rl)
        assert m.mdeos_plan(s, skin).ext_cap == p.ext_cap


def test_multi_image_flagged():
    p = m.mdeos_plan(spec(rho=1.2, n_c=3, rc=3.0))
    assert p.multi_image == 1
    assert m.mdeos_plan(spec()).multi_image == 0


def test_cell_bytes():
    assert m.mdeos_cell_bytes(5) >= 500 * 48


def test_create_without_device_fails_cleanly():
    if m.mdeos_device_count() > 0:
        pytest.skip("a device is present")
    with pytest.raises(m.MdeosError) as e:
        m.mdeos_create()
    assert e.value.status == m.NO_DEVICE


def test_create_rejects_unknown_precision():
    # checked before any device call, so this runs on the CPU too
    with pytest.raises(m.MdeosError) as e:
        m.mdeos_create(precision=7)
    assert e.value.status == m.INVALID_ARG
    assert "precision" in str(e.value)


@pytest.mark.parametrize("kw,what", [({"potential": 2}, "potential"), ({"potential": 1, "eam_c": float("nan")},
                                                                        "eam_c"),
                                     ({"prune_skin": float("nan")}, "prune_skin"),
                                     ({"prune_skin": float("inf")}, "prune_skin")])
def test_create_rejects_an_unknown_potential(kw, what):
    # checked before any device call, so this runs on the CPU too
    with pytest.raises(m.MdeosError) as e:
        m.mdeos_create(**kw)
    assert e.value.status == m.INVALID_ARG
    assert what in str(e.value)


def test_eam_workload_cells_plan_into_eam_shapes():
    """Every cell of the embedded-atom bench workload plans (at skins 0.15 and
    0.25, and at the embedded-atom default of 0.5) with at most 4095 position slots, which the
    4096-stride embedded-atom shapes for 500-atom boxes hold (a shape serves any plan it covers)."""
    from paper_2508_06012_amd import workloads as wl
    w = wl.eam_cu()
    assert w.potential == 1 and w.n == 4096 and set(w.N) == {500}
    assert 4.0 <= w.rho.min() and w.rho.max() <= 6.0
    specs, _ = m.specs_from_workload(w.subset(np.arange(0, 4096, 64)))
    caps = [m.mdeos_plan(s, skin).ext_cap for s in specs for skin in (0.15, 0.25, 0.5)]
    assert max(caps) < 4096, max(caps)


def test_config_layout_matches_header():
    """The binding's config struct lists the header's fields in order."""
    import re
    hdr = open(os.path.join(ROOT, "include", "mdeos.h")).read()
    end = hdr.index("} mdeos_config;")
    body = hdr[hdr.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    names = re.findall(r"\b(\w+);", re.sub(r"/\*.*?\*/", "", body, flags=re.S))
    assert names == [f[0] for f in m.Config._fields_]


def test_schedule_layout_matches_header():
    hdr = open(os.path.join(ROOT, "include", "mdeos.h")).read()
    end = hdr.index("} mdeos_schedule;")
    body = hdr[hdr.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    names = re.findall(r"\b(\w+)(?:\[\w+\])?;", re.sub(r"/\*.*?\*/", "", body, flags=re.S))
    assert names == [f[0] for f in m.Schedule._fields_]


@pytest.mark.parametrize("ensemble,gamma,ok", [(0, 0.0, True), (1, 1.0, True), (1, 0.0, True), (2, 1.0, False),
                                               (1, -0.5, False), (1, float("nan"), False)])
def test_validate_ensemble_and_friction(ensemble, gamma, ok):
    spec = m.make_specs(0.8, 1.5, 4, 2.5, 0.005, 1, 0)[0]
    sch = m.make_schedule(100, 50, (10,), ensemble=ensemble, gamma=gamma)
    st = m.lib().mdeos_validate(C.byref(spec), C.byref(sch))
    assert (st == m.OK) == ok


GUARD_CHILD = r"""
import ctypes, sys
sys.path.insert(0, sys.argv[1])
from paper_2508_06012_amd import mdeos as m
ctypes.CDLL(m.LIB_PATH)  # the library first: it maps the system HIP runtime
import torch  # then torch maps its own copy
class S:
    cuda_stream = 0
print("runtimes", len(m.hip_runtimes()))
try:
    m._stream(S())
    print("accepted")
except m.MdeosError as e:
    print("refused:", e)
"""


def test_torch_stream_refused_under_two_hip_runtimes():
    """A process that loaded the library before torch maps two HIP runtimes;
    the binding then refuses a torch stream instead of handing the library a
    handle of the other runtime (checked in a child process, no device)."""
    pytest.importorskip("torch")
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", GUARD_CHILD, root], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    if "runtimes 1" in r.stdout:
        pytest.skip("torch resolved the library's runtime: one runtime mapped")
    assert "runtimes 2" in r.stdout and "refused: " in r.stdout, r.stdout
