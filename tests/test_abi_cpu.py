"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every function include/coulomb.h declares, sizes workspaces, keeps launch
configurations, and rejects bad arguments before enqueueing anything (every
call below fails validation, so no kernel is ever launched)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def api():
    from paper_2106_11143_amd import api as A
    if not os.path.exists(A.LIB_PATH):
        from paper_2106_11143_amd import build
        build.build(verbose=False)
    A.lib()
    return A


def header_functions():
    src = open(os.path.join(ROOT, "include", "coulomb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_function(api):
    names = header_functions()
    assert {"coulomb_forces", "coulomb_energy", "md_step", "md_run", "coulomb_hvp"} <= set(names)
    L = api.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(api.EXPORTS) == set(names)


def test_workspace_sizes(api):
    L = api.lib()
    assert L.cb_workspace_size(0, 0, 1, 1, 0) == 0
    assert L.cb_workspace_size(0, 10, 1, 1, 9) == 0
    assert L.cb_workspace_size(4, 10, 1, 9, 0) == 0
    f = L.cb_workspace_size(0, 100000, 1, 1, 0)
    assert f >= 64 * 3 * 100000 * 8
    assert L.cb_workspace_size(4, 1000, 1, 4, 0) >= 64 * 12 * 1000 * 8
    assert L.cb_workspace_size(3, 10000, 16, 1, 0) < L.cb_workspace_size(3, 10000, 1, 1, 0)


def test_config_roundtrip(api):
    api.set_config("forces", 5000, "mixed", p=2, wg=128, splits=7)
    c = api.get_config("forces", 4500, "mixed")  # same power-of-two bucket
    assert (c["p"], c["wg"], c["splits"], c["tuned"]) == (2, 128, 7, True)
    d = api.get_config("forces", 5000, "fp64")
    assert not d["tuned"]
    with pytest.raises(api.CoulombError) as e:
        api.set_config("forces", 5000, "fp64", p=3, wg=256, splits=1)
    assert e.value.status == api.CB_EINVAL
    with pytest.raises(api.CoulombError):
        api.set_config("hvp", 5000, "fp64", p=4, wg=256, splits=1)
    with pytest.raises(api.CoulombError):
        api.set_config("forces", 5000, "fp64", p=1, wg=256, splits=65)


def _ws():
    return C.c_void_p(1 << 20)  # never dereferenced: every call below fails validation first


def test_forces_argument_errors(api):
    L = api.lib()
    P = C.c_void_p(1 << 21)
    big = 1 << 40
    # n out of range
    assert L.coulomb_forces(0, P, P, P, P, 0.0, 0, P, P, P, _ws(), big, None) == api.CB_EINVAL
    assert "n = 0" in api.last_error()
    # bad precision, bad eps2
    assert L.coulomb_forces(10, P, P, P, P, 0.0, 7, P, P, P, _ws(), big, None) == api.CB_EINVAL
    assert L.coulomb_forces(10, P, P, P, P, -1.0, 0, P, P, P, _ws(), big, None) == api.CB_EINVAL
    assert L.coulomb_forces(10, P, P, P, P, float("nan"), 0, P, P, P, _ws(), big, None) == api.CB_EINVAL
    # workspace problems
    assert L.coulomb_forces(10, P, P, P, P, 0.0, 0, P, P, P, None, big, None) == api.CB_EINVAL
    assert L.coulomb_forces(10, P, P, P, P, 0.0, 0, P, P, P, C.c_void_p((1 << 20) + 8), big, None) == api.CB_EINVAL
    assert L.coulomb_forces(10, P, P, P, P, 0.0, 0, P, P, P, _ws(), 100, None) == api.CB_ENOWS
    assert "workspace" in api.last_error()
    # NULL arrays and aliasing
    assert L.coulomb_forces(10, None, P, P, P, 0.0, 0, P, P, P, _ws(), big, None) == api.CB_EINVAL
    a, b = C.c_void_p(1 << 22), C.c_void_p((1 << 22) + 40)
    o1, o2, o3 = C.c_void_p(1 << 23), C.c_void_p(1 << 24), C.c_void_p(1 << 25)
    assert L.coulomb_forces(10, a, o1, o1, o1, 0.0, 0, b, o2, o3, _ws(), big, None) == api.CB_EINVAL
    assert "alias" in api.last_error()


def test_forces_range_argument_errors(api):
    L = api.lib()
    P = C.c_void_p(1 << 21)
    big = 1 << 40
    for i0, i1 in ((-1, 5), (5, 5), (6, 5), (0, 11)):
        assert L.coulomb_forces_range(10, i0, i1, P, P, P, P, 0.0, 0, P, P, P, _ws(), big, None) == api.CB_EINVAL
        assert "i0" in api.last_error()
    assert L.coulomb_forces_range(10, 0, 5, P, P, P, P, 0.0, 0, None, P, P, _ws(), big, None) == api.CB_EINVAL
    assert L.coulomb_forces_range(10, 0, 5, P, P, P, P, 0.0, 0, P, P, P, _ws(), 100, None) == api.CB_ENOWS
    # an output of i1 - i0 doubles inside an input array is rejected
    x = C.c_void_p(1 << 22)
    o = C.c_void_p((1 << 22) + 8 * 9)
    o2, o3 = C.c_void_p(1 << 23), C.c_void_p(1 << 24)
    assert L.coulomb_forces_range(10, 0, 2, x, P, P, P, 0.0, 0, o, o2, o3, _ws(), big, None) == api.CB_EINVAL
    assert "alias" in api.last_error()


def test_md_argument_errors(api):
    L = api.lib()
    big = 1 << 40
    arrs = [C.c_void_p((k + 1) << 24) for k in range(11)]
    s = api.State(*arrs[:9])
    q, m = arrs[9], arrs[10]
    tr = api.make_trap(dict(kind=0, wx=1e6, wy=1e6, wz=1e5))
    # dt <= 0
    assert L.md_step(10, C.byref(s), q, m, C.byref(tr), 0.0, 0.0, 0.0, 0, _ws(), big, None) == api.CB_EINVAL
    # negative friction
    tg = api.make_trap(dict(kind=0, wx=1e6, wy=1e6, wz=1e5, gamma=-1e-20))
    assert L.md_step(10, C.byref(s), q, m, C.byref(tg), 0.0, 1e-9, 0.0, 0, _ws(), big, None) == api.CB_EINVAL
    assert "gamma" in api.last_error()
    # the adjoint step is friction-free only
    tf = api.make_trap(dict(kind=0, wx=1e6, wy=1e6, wz=1e5, gamma=1e-20))
    lam, dl = C.c_void_p(1 << 31), C.c_void_p(1 << 32)
    assert L.md_adjoint_step(10, arrs[0], arrs[1], arrs[2], q, m, C.byref(tf), 1e-9, 0.0, 0, 0, lam, dl, _ws(), big,
                             None) == api.CB_EUNSUPPORTED
    assert "friction" in api.last_error()
    # non-finite trap, bad kind
    tn = api.make_trap(dict(kind=0, wx=float("inf")))
    assert L.md_step(10, C.byref(s), q, m, C.byref(tn), 0.0, 1e-9, 0.0, 0, _ws(), big, None) == api.CB_EINVAL
    tk = api.make_trap(dict(kind=3))
    assert L.md_step(10, C.byref(s), q, m, C.byref(tk), 0.0, 1e-9, 0.0, 0, _ws(), big, None) == api.CB_EINVAL
    # overlapping state arrays
    s2 = api.State(*([arrs[0]] * 9))
    assert L.md_step(10, C.byref(s2), q, m, C.byref(tr), 0.0, 1e-9, 0.0, 0, _ws(), big, None) == api.CB_EINVAL
    # md_run: offsets not increasing / not starting at 0, every < 1 with energies
    offs = (C.c_int64 * 3)(0, 5, 5)
    trs = (api.Trap * 2)(tr, tr)
    assert L.md_run(2, offs, C.byref(s), q, m, trs, 0.0, 1e-9, 10, 0.0, 0, 1, None, 0, _ws(), big, None) == api.CB_EINVAL
    offs = (C.c_int64 * 2)(1, 5)
    assert L.md_run(1, offs, C.byref(s), q, m, trs, 0.0, 1e-9, 10, 0.0, 0, 1, None, 0, _ws(), big, None) == api.CB_EINVAL
    offs = (C.c_int64 * 2)(0, 10)
    en = C.c_void_p(1 << 30)
    assert L.md_run(1, offs, C.byref(s), q, m, trs, 0.0, 1e-9, 10, 0.0, 0, 1, en, 0, _ws(), big, None) == api.CB_EINVAL
    assert L.md_run(1, offs, C.byref(s), q, m, trs, 0.0, 1e-9, 10, 0.0, 0, 8, None, 0, _ws(), big, None) == api.CB_EINVAL


def test_poll_flags_rejects_null(api):
    assert api.lib().cb_poll_flags(None, None) == api.CB_EINVAL


def test_batched_rejects_runs_beyond_lds_limit(api):
    L = api.lib()
    arrs = [C.c_void_p((k + 1) << 26) for k in range(11)]
    s = api.State(*arrs[:9])
    tr = api.make_trap(dict(kind=0, wx=1e6, wy=1e6, wz=1e5))
    offs = (C.c_int64 * 3)(0, 100, 100 + 4097)
    trs = (api.Trap * 2)(tr, tr)
    st = L.md_run(2, offs, C.byref(s), arrs[9], arrs[10], trs, 0.0, 1e-9, 10, 0.0, 0, 1, None, 0, _ws(), 1 << 40, None)
    assert st == api.CB_EUNSUPPORTED
    assert "4096" in api.last_error()


def test_load_tuning_missing_file_and_foreign_arch(api, tmp_path):
    api.load_tuning(str(tmp_path / "missing.jsonl"))  # a missing cache is not an error
    p = tmp_path / "cache.jsonl"
    p.write_text('{"arch": "gfx000", "op": 0, "prec": 0, "bucket": 12, "n": 4000, "p": 2, "wg": 128, '
                 '"splits": 9, "ms": 1.0}\nnot json\n')
    api.load_tuning(str(p))  # entries of another architecture are ignored
    assert not api.get_config("forces", 4000, "fp64")["tuned"]


def test_symmetric_config_validation(api):
    api.set_config("md_run", 50000, "fp64", p=3, wg=4, splits=2048, algo=1)
    c = api.get_config("md_run", 50000, "fp64")
    assert (c["algo"], c["p"], c["wg"], c["splits"], c["tuned"]) == (1, 3, 4, 2048, True)
    api.reset_config("md_run", 50000, "fp64")
    assert api.get_config("md_run", 50000, "fp64")["algo"] == 2  # the default at this size
    c = api.get_config("md_run", 250, "fp64")  # small runs: one launch per step
    assert (c["algo"], c["p"], c["wg"], c["splits"], c["tuned"]) == (3, 1, 64, 7, False)
    assert api.get_config("forces", 250, "fp64")["algo"] == 0
    assert (api.get_config("md_run", 256, "fp64")["algo"], api.get_config("md_run", 257, "fp64")["algo"]) == (3, 0)
    assert api.get_config("md_run", 300, "fp64")["splits"] == 18  # j-ranges of 16
    c = api.get_config("md_run", 1024, "fp64")  # two launches, j-ranges of 16 ions up to 4096
    assert (c["algo"], c["wg"], c["splits"]) == (0, 256, 64)
    assert api.get_config("md_run", 512, "fp64")["splits"] == 32
    assert api.get_config("md_step", 4096, "fp64")["splits"] == 64
    assert api.get_config("md_run", 8192, "fp64")["splits"] == 32  # ranges of 64 beyond
    assert api.get_config("forces", 1024, "fp64")["splits"] == 32  # the forces keep ranges of 32
    assert api.get_config("md_run", 1000, "fp64")["algo"] == 0
    assert api.get_config("md_run", 10000, "fp64")["algo"] == 0
    api.set_config("md_step", 8192, "fp64", p=1, wg=64, splits=7, algo=3)
    assert api.get_config("md_step", 8192, "fp64")["splits"] == 7
    api.reset_config("md_step", 8192, "fp64")
    for bad in (dict(op="forces", n=1000, p=1, wg=64, splits=8),  # md_step / md_run only
                dict(op="md_run", n=8193, p=1, wg=64, splits=8),  # beyond the small-run limit
                dict(op="md_run", n=1000, p=1, wg=64, splits=33),
                dict(op="md_run", n=1000, p=2, wg=64, splits=8)):
        with pytest.raises(api.CoulombError):
            api.set_config(bad["op"], bad["n"], "fp64", p=bad["p"], wg=bad["wg"], splits=bad["splits"], algo=3)
    # the energy takes the Newton's-third-law stage too (the potential as a fourth component)
    assert api.get_config("energy", 50000, "fp64")["algo"] == 2
    # row-group tiles from 81920 ions (P = 8, JL = 512), one-wave tiles below
    for op in ("forces", "energy", "md_step", "md_run"):
        c = api.get_config(op, 100000, "fp64")
        assert (c["algo"], c["p"], c["wg"], c["splits"]) == (4, 8, 4, 512)
        assert api.get_config(op, 81919, "fp64")["algo"] == 2
        assert api.get_config(op, 81920, "fp64")["algo"] == 4
        assert api.get_config(op, 262144, "fp64")["algo"] == 4
        assert api.get_config(op, 262145, "fp64")["algo"] == 0
    assert api.get_config("energy", 10000, "fp64")["algo"] == 0
    for algo in (1, 2):
        for p in (2, 3, 4, 5, 6, 8):
            for jl in (256, 512, 1024, 2048):
                api.set_config("forces", 5000, "fp64", p=p, wg=4, splits=jl, algo=algo)
                c = api.get_config("forces", 5000, "fp64")
                assert (c["algo"], c["p"], c["splits"]) == (algo, p, jl)
    api.reset_config("forces", 5000, "fp64")
    with pytest.raises(api.CoulombError):
        api.set_config("forces", 5000, "fp64", p=4, wg=4, splits=512, algo=3)
    for bad in (dict(op="forces", n=1 << 19, p=2, wg=4, splits=1024),  # beyond the symmetric size limit
                dict(op="hvp", n=5000, p=2, wg=4, splits=1024),  # not a segment length of the HVP tiles
                dict(op="adjoint", n=5000, p=2, wg=4, splits=1024),
                dict(op="forces", n=5000, p=4, wg=8, splits=1024),  # groups are 4 j's
                dict(op="forces", n=5000, p=7, wg=4, splits=1024),
                dict(op="forces", n=5000, p=1, wg=4, splits=1024),
                dict(op="forces", n=5000, p=2, wg=4, splits=128),
                dict(op="forces", n=5000, p=2, wg=4, splits=1000)):
        with pytest.raises(api.CoulombError):
            api.set_config(bad["op"], bad["n"], "fp64", p=bad["p"], wg=bad["wg"], splits=bad["splits"], algo=2)
        with pytest.raises(api.CoulombError):
            api.set_config(bad["op"], bad["n"], "fp64", p=bad["p"], wg=bad["wg"], splits=bad["splits"], algo=1)


def test_fp32_displacement_ablation_is_forces_only(api):
    L = api.lib()
    big = 1 << 40
    P = C.c_void_p(1 << 21)
    assert L.cb_workspace_size(0, 100, 1, 1, 4) > 0
    assert L.cb_workspace_size(0, 100, 1, 1, 5) == 0
    assert L.coulomb_energy(10, P, P, P, P, 0.0, 4, P, _ws(), big, None) == api.CB_EUNSUPPORTED
    arrs = [C.c_void_p((k + 1) << 24) for k in range(11)]
    s = api.State(*arrs[:9])
    tr = api.make_trap(dict(kind=0, wx=1e6, wy=1e6, wz=1e5))
    assert L.md_step(10, C.byref(s), arrs[9], arrs[10], C.byref(tr), 0.0, 1e-9, 0.0, 4, _ws(), big,
                     None) == api.CB_EUNSUPPORTED
    offs = (C.c_int64 * 2)(0, 10)
    assert L.md_run(1, offs, C.byref(s), arrs[9], arrs[10], C.byref(tr), 0.0, 1e-9, 5, 0.0, 4, 1, None, 0, _ws(),
                    big, None) == api.CB_EUNSUPPORTED
    v = C.c_void_p(1 << 30)
    assert L.coulomb_hvp(10, P, P, P, P, 1, v, C.c_void_p(1 << 31), None, None, 0.0, 0.0, 4, _ws(), big,
                         None) == api.CB_EUNSUPPORTED
    assert L.cb_autotune(0, 1000, 4, None) == api.CB_EUNSUPPORTED


def test_ensemble_config_validation_and_workspace(api):
    """The ensemble path key of md_run with several runs: default, the two
    valid shapes, rejections; the md_run workspace covers the stepped path
    (about 0.5 KB per ion for any split into runs of at most 4096)."""
    c = api.get_config("md_ensemble", 1_000_000, "fp64")
    assert (c["algo"], c["p"], c["wg"], c["splits"], c["tuned"]) == (2, 4, 4, 256, False)
    api.set_config("md_ensemble", 1_000_000, "fp64", p=4, wg=512, splits=1, algo=0)
    c = api.get_config("md_ensemble", 1_000_000, "fp64")
    assert (c["algo"], c["tuned"]) == (0, True)
    for p in (4, 8):
        for jl in (256, 512):
            api.set_config("md_ensemble", 1_000_000, "mixed", p=p, wg=4, splits=jl, algo=2)
            c = api.get_config("md_ensemble", 1_000_000, "mixed")
            assert (c["algo"], c["p"], c["splits"], c["tuned"]) == (2, p, jl, True)
    api.reset_config("md_ensemble", 1_000_000, "fp64")
    api.reset_config("md_ensemble", 1_000_000, "mixed")
    assert not api.get_config("md_ensemble", 1_000_000, "mixed")["tuned"]
    for bad in (dict(p=2, wg=4, splits=256, algo=2), dict(p=4, wg=4, splits=1024, algo=2),
                dict(p=4, wg=4, splits=256, algo=1), dict(p=4, wg=256, splits=1, algo=0),
                dict(p=1, wg=512, splits=1, algo=0), dict(p=8, wg=8, splits=512, algo=2)):
        with pytest.raises(api.CoulombError):
            api.set_config("md_ensemble", 1_000_000, "fp64", **bad)
    assert api.lib().cb_workspace_size(6, 1000, 2, 1, 0) == 0  # a configuration key, not a call
    for ntot, nrun in ((1_070_000, 512), (8192, 2), (5000, 100)):
        ws = api.workspace_size("md_run", ntot, nrun=nrun)
        assert 400 * ntot <= ws <= 1000 * ntot + (1 << 24), (ntot, nrun, ws)


def test_trap_constants_match_oracle(api, oracle):
    """cb_trap_k (host; the same function the kernels evaluate) against the
    oracle's trap constants: RF drive with a DC term and a phase, a ramp
    before, inside and after its ramp, a static trap."""
    cases = [(dict(kind=1, rf_a=0.02, rf_q=0.3, rf_omega=6.283e7, rf_phase=0.7, wz=6.283e5), t)
             for t in (0.0, 3.7e-8, 1.01e-6)]
    ramp = dict(kind=0, wx=9.42e6, wy=9.0e6, wz=9.42e5, wx1=3.77e6, wy1=3.5e6, t_ramp0=1e-6, t_ramp1=21e-6)
    cases += [(ramp, t) for t in (0.0, 1e-6, 7.3e-6, 21e-6, 1.0)]
    cases += [(dict(kind=0, wx=6.283e6, wy=5.0e6, wz=1.2566e6), 0.0), (dict(kind=1, rf_q=0.25, rf_omega=4.4e7,
                                                                            rf_phase=-2.0, wz=1e6), 2.2e-7)]
    for trap, t in cases:
        k = np.array(api.trap_k(trap, t))
        ref = oracle.trap_k(trap, t)
        assert np.all(np.abs(k - ref) <= 4 * 2.0 ** -53 * np.abs(ref)), (trap, t, k, ref)
    with pytest.raises(api.CoulombError):
        api.trap_k(dict(kind=2), 0.0)
    with pytest.raises(api.CoulombError):
        api.trap_k(dict(kind=0, wx=float("nan")), 0.0)


def test_trap_grad_argument_errors(api):
    L = api.lib()
    big = 1 << 40
    P = C.c_void_p(1 << 21)
    x, y, z, q, m = (C.c_void_p((k + 1) << 24) for k in range(5))
    g1, g2, g3, u = (C.c_void_p((k + 8) << 24) for k in range(4))
    tr = api.make_trap(dict(kind=0, wx=1e6, wy=1e6, wz=1e5))
    call = lambda *a: L.coulomb_trap_grad(*a)
    assert L.cb_workspace_size(7, 1000, 1, 1, 0) >= L.cb_workspace_size(1, 1000, 1, 1, 0)
    assert call(0, x, y, z, q, m, C.byref(tr), 0.0, 0.0, 0, g1, g2, g3, u, _ws(), big, None) == api.CB_EINVAL
    assert call(10, None, y, z, q, m, C.byref(tr), 0.0, 0.0, 0, g1, g2, g3, u, _ws(), big, None) == api.CB_EINVAL
    # the gradient's three rows together or not at all, and something to do
    assert call(10, x, y, z, q, m, C.byref(tr), 0.0, 0.0, 0, g1, None, g3, u, _ws(), big, None) == api.CB_EINVAL
    assert call(10, x, y, z, q, m, C.byref(tr), 0.0, 0.0, 0, None, None, None, None, _ws(), big, None) == api.CB_EINVAL
    assert "nothing" in api.last_error()
    # with m the trap is checked; without it the trap is ignored
    bad = api.make_trap(dict(kind=5))
    assert call(10, x, y, z, q, m, C.byref(bad), 0.0, 0.0, 0, g1, g2, g3, u, _ws(), big, None) == api.CB_EINVAL
    assert call(10, x, y, z, q, m, None, 0.0, 0.0, 0, g1, g2, g3, u, _ws(), big, None) == api.CB_EINVAL
    assert call(10, x, y, z, q, m, C.byref(tr), float("inf"), 0.0, 0, g1, g2, g3, u, _ws(), big, None) == api.CB_EINVAL
    # aliasing, precision, workspace
    assert call(10, x, y, z, q, m, C.byref(tr), 0.0, 0.0, 0, x, g2, g3, u, _ws(), big, None) == api.CB_EINVAL
    assert call(10, x, y, z, q, m, C.byref(tr), 0.0, 0.0, 0, g1, g2, g3, C.c_void_p((8 << 24) + 16), _ws(), big,
                None) == api.CB_EINVAL
    assert call(10, x, y, z, q, m, C.byref(tr), 0.0, 0.0, 4, g1, g2, g3, u, _ws(), big, None) == api.CB_EUNSUPPORTED
    assert call(10, x, y, z, q, m, C.byref(tr), 0.0, 0.0, 0, g1, g2, g3, u, _ws(), 100, None) == api.CB_ENOWS


def test_noalloc_argument_errors(api):
    """coulomb_forces_noalloc validates before it touches a device: sizes
    beyond its static scratch, bad n, precision, eps2, NULL and aliasing."""
    L = api.lib()
    P = C.c_void_p(1 << 21)
    o1, o2, o3 = C.c_void_p(1 << 23), C.c_void_p(1 << 24), C.c_void_p(1 << 25)
    assert L.coulomb_forces_noalloc(2796203, P, P, P, P, 0.0, 0, o1, o2, o3, None) == api.CB_ENOWS
    assert "scratch" in api.last_error()
    assert L.coulomb_forces_noalloc(0, P, P, P, P, 0.0, 0, o1, o2, o3, None) == api.CB_EINVAL
    assert L.coulomb_forces_noalloc(10, P, P, P, P, 0.0, 9, o1, o2, o3, None) == api.CB_EINVAL
    assert L.coulomb_forces_noalloc(10, P, P, P, P, -1.0, 0, o1, o2, o3, None) == api.CB_EINVAL
    assert L.coulomb_forces_noalloc(10, None, P, P, P, 0.0, 0, o1, o2, o3, None) == api.CB_EINVAL
    assert L.coulomb_forces_noalloc(10, o1, P, P, P, 0.0, 0, o1, o2, o3, None) == api.CB_EINVAL
    assert "alias" in api.last_error()
    assert L.coulomb_forces_noalloc(10, P, P, P, P, 0.0, 0, o1, o1, o3, None) == api.CB_EINVAL


def test_hvp_config_validation(api):
    """The Newton's-third-law HVP shapes (algorithm 2): p in {1, 2, 4}, wg =
    the most vectors per pass in {1, 2, 4}, segments of 64 .. 512, n up to
    131072 p; for the HVP and the adjoint step."""
    for op in ("hvp", "adjoint"):
        for p in (1, 2, 4):
            for wg in (1, 2, 4):
                for jl in (64, 128, 256, 512):
                    api.set_config(op, 5000, "fp64", p=p, wg=wg, splits=jl, algo=2)
                    c = api.get_config(op, 5000, "fp64")
                    assert (c["algo"], c["p"], c["wg"], c["splits"]) == (2, p, wg, jl)
        api.reset_config(op, 5000, "fp64")
        for bad in (dict(p=3, wg=4, splits=128), dict(p=2, wg=3, splits=128), dict(p=2, wg=4, splits=1024),
                    dict(p=2, wg=4, splits=96)):
            with pytest.raises(api.CoulombError):
                api.set_config(op, 5000, "fp64", algo=2, **bad)
        with pytest.raises(api.CoulombError):  # beyond the tile table of p = 1
            api.set_config(op, 131073, "fp64", p=1, wg=4, splits=128, algo=2)
        api.set_config(op, 131073, "fp64", p=2, wg=4, splits=128, algo=2)
        api.reset_config(op, 131073, "fp64")


def test_row_group_config_validation(api):
    """Algorithm 4 (four i-blocks per workgroup): forces, energy and md
    calls, p in {4, 6, 8}, segments of the symmetric path, n <= 2^18; its
    workspace holds a kSymRows-th of the reaction partials."""
    for op in ("forces", "energy", "md_step", "md_run"):
        api.set_config(op, 50000, "fp64", p=8, wg=4, splits=512, algo=4)
        c = api.get_config(op, 50000, "fp64")
        assert (c["algo"], c["p"], c["wg"], c["splits"], c["tuned"]) == (4, 8, 4, 512, True)
        api.reset_config(op, 50000, "fp64")
    for bad in (dict(op="forces", n=50000, p=2, splits=512),   # p outside {4, 6, 8}
                dict(op="forces", n=50000, p=8, splits=384),   # not a segment length
                dict(op="forces", n=300000, p=8, splits=512),  # beyond 2^18
                dict(op="hvp", n=8192, p=4, splits=128),       # forces-shaped calls only
                dict(op="md_ensemble", n=50000, p=4, splits=256)):
        with pytest.raises(api.CoulombError):
            api.set_config(bad["op"], bad["n"], "fp64", p=bad["p"], wg=4, splits=bad["splits"], algo=4)
    n = 100000
    sizes = {}
    for algo in (2, 4):
        api.set_config("forces", n, "fp64", p=8, wg=4, splits=512, algo=algo)
        try:
            sizes[algo] = api.workspace_size("forces", n)
        finally:
            api.reset_config("forces", n, "fp64")
    # R shrinks fourfold (234 -> 59 MB at N = 1e5); Pi and the tile table stay
    assert 0 < sizes[4] < sizes[2] - 150e6
