"""Parity of the headline workload at full size (cloud100k, N = 1e5) on the
default launch (the Newton's-third-law force stage): forces on every ion,
a two-step velocity-Verlet run on every ion within the oracle's round-off
envelope, and bitwise repeatability of the force stage.

The oracle work (seven all-pairs evaluations at N = 1e5, compensated sums)
is done once per module and takes about a minute on 16 host cores."""
import numpy as np
import pytest

from paper_2106_11143_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

NSTEPS = 2


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_11143_amd import api as A
    A.lib()
    return A


@pytest.fixture(scope="module")
def ref100k(oracle):
    """Oracle forces (with kappa) on every ion, and a two-step run from the
    workload's start with the same run in reversed ion order (its round-off
    envelope)."""
    import time
    d = inputs.cloud100k()
    t0 = time.perf_counter()
    fx, fy, fz, kappa = oracle.forces(d["x"], d["y"], d["z"], d["q"], kappa=True)
    print(f"[oracle] forces on all {d['n']} ions: {time.perf_counter() - t0:.1f} s", flush=True)
    st = inputs.state9(d)
    t0 = time.perf_counter()
    ref, _, _ = oracle.md_run(st, d["q"], d["m"], d["trap"], 0.0, d["dt"], NSTEPS)
    perm = np.arange(d["n"])[::-1]
    alt, _, _ = oracle.md_run(st[:, perm], d["q"][perm], d["m"][perm], d["trap"], 0.0, d["dt"], NSTEPS)
    alt = alt[:, np.argsort(perm)]
    print(f"[oracle] two {NSTEPS}-step runs: {time.perf_counter() - t0:.1f} s", flush=True)
    return d, np.stack([fx, fy, fz]), kappa, ref, alt


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cloud100k_forces_every_ion(api, ref100k, prec):
    """coulomb_forces at N = 1e5 in the default launch against the oracle on
    all 100000 ions (per-ion relative error: 1e-12 for FP64, 1e-7 for mixed)."""
    from _gpu_util import dev, host, per_ion_rel, report
    d, F_ref, kappa, _, _ = ref100k
    cfg = api.get_config("forces", d["n"], prec)
    assert cfg["algo"] in (1, 2, 4)  # the default at this size is the Newton's-third-law stage
    F = np.stack([host(t) for t in api.coulomb_forces(*(dev(d[k]) for k in "xyzq"), prec=prec)])
    err = per_ion_rel(F, F_ref)
    report(f"cloud100k/{prec} all ions", err, kappa)
    assert err.max() <= (1e-12 if prec == "fp64" else 1e-7)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cloud100k_md_run_every_ion_within_envelope(api, ref100k, prec):
    """A two-step md_run of the headline workload on the default path: every
    ion's position, velocity and acceleration against the oracle run, within
    ten times the oracle's own round-off envelope (its reversed-order run)
    plus the precision's bound (per ion for the acceleration, on the block's
    scale for positions and velocities)."""
    from _gpu_util import dev, state_host, state_tensors
    d, _, _, ref, alt = ref100k
    tol = 1e-12 if prec == "fp64" else 1e-7
    ts = state_tensors(inputs.state9(d))
    api.md_run(ts, dev(d["q"]), dev(d["m"]), d["trap"], 0.0, d["dt"], NSTEPS, prec=prec)
    got = state_host(ts)
    for blk in (slice(0, 3), slice(3, 6)):
        D = np.abs(alt[blk] - ref[blk]).max()
        err = np.abs(got[blk] - ref[blk]).max()
        scale = np.abs(ref[blk]).max()
        print(f"[cloud100k md {prec}] block {blk}: err={err:.3e} envelope={D:.3e} scale={scale:.3e}", flush=True)
        assert err <= 10 * D + tol * 0.1 * scale
    # accelerations ion by ion: |da_i| <= 10 |envelope_i| + tol |a_i|
    a_ref, a_alt, a_got = ref[6:9], alt[6:9], got[6:9]
    dev_i = np.linalg.norm(a_got - a_ref, axis=0)
    env_i = np.linalg.norm(a_alt - a_ref, axis=0)
    nrm_i = np.linalg.norm(a_ref, axis=0)
    ratio = dev_i / (10 * env_i + tol * nrm_i)
    worst = int(np.argmax(ratio))
    print(f"[cloud100k md {prec}] accel: max rel {np.max(dev_i / nrm_i):.3e}, worst ion {worst} at "
          f"{ratio[worst]:.3f} of its bound", flush=True)
    assert ratio.max() <= 1.0
    assert api.poll_flags() == 0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cloud100k_force_stage_is_bitwise_repeatable(api, prec):
    """The default force stage at N = 1e5 (tiles, reactions, fixed-order
    finish; no atomics) gives bitwise identical forces on repeated calls,
    and md_run repeats bitwise too."""
    import torch
    from _gpu_util import dev, state_tensors
    d = inputs.cloud100k()
    args = [dev(d[k]) for k in "xyzq"]
    a = [t.clone() for t in api.coulomb_forces(*args, prec=prec)]
    for _ in range(2):
        b = api.coulomb_forces(*args, prec=prec)
        for u, v in zip(a, b):
            assert torch.equal(u, v)
    st = inputs.state9(d)
    runs = []
    for _ in range(2):
        ts = state_tensors(st)
        api.md_run(ts, dev(d["q"]), dev(d["m"]), d["trap"], 0.0, d["dt"], 3, prec=prec)
        runs.append(torch.stack(ts))
    assert torch.equal(runs[0], runs[1])


@pytest.mark.parametrize("algo,p,jl", [(2, 8, 512), (4, 8, 512)])
def test_cloud100k_symmetric_variants_agree_and_repeat(api, oracle, algo, p, jl):
    """Both Newton's-third-law variants at N = 1e5 (one wave per tile; four
    i-blocks per workgroup): bitwise repeatable, within the tolerance of the
    oracle on sampled ions, and within rounding of each other."""
    import torch
    from _gpu_util import dev, per_ion_rel
    d = inputs.group_by_charge(inputs.cloud100k())
    n = d["n"]
    args = [dev(d[k]) for k in "xyzq"]
    idx = np.sort(np.random.Generator(np.random.PCG64(77)).choice(n, 300, replace=False))
    ref = np.stack(oracle.forces(d["x"], d["y"], d["z"], d["q"], idx=idx))
    api.set_config("forces", n, "fp64", p=p, wg=4, splits=jl, algo=algo)
    try:
        a = [t.clone() for t in api.coulomb_forces(*args)]
        b = api.coulomb_forces(*args)
    finally:
        api.reset_config("forces", n, "fp64")
    for u, v in zip(a, b):
        assert torch.equal(u, v)
    F = np.stack([t.cpu().numpy() for t in a])
    assert per_ion_rel(F[:, idx], ref).max() <= 1e-12
    dflt = np.stack([t.cpu().numpy() for t in api.coulomb_forces(*args)])
    assert per_ion_rel(F, dflt).max() <= 1e-13


def test_cloud100k_energy_on_the_default_stage(api, oracle):
    """coulomb_energy of the headline system (N = 1e5) in the default launch,
    the row-group tiles with the pair energies summed in the tiles and each
    ion's share added by the finish, in the seeded order and grouped by
    charge, against the oracle's compensated U_C."""
    from _gpu_util import dev
    d = inputs.cloud100k()
    assert api.get_config("energy", d["n"], "fp64")["algo"] == 4
    ref, _ = oracle.coulomb_energy(d["x"], d["y"], d["z"], d["q"])
    for order, dd in (("seeded", d), ("grouped", inputs.group_by_charge(d))):
        for prec, tol in (("fp64", 1e-12), ("mixed", 1e-9)):
            u = float(api.coulomb_energy(*(dev(dd[k]) for k in "xyzq"), prec=prec)[0])
            print(f"[cloud100k energy {order} {prec}] rel err {abs(u - ref) / abs(ref):.3e}", flush=True)
            assert abs(u - ref) <= tol * abs(ref), (order, prec, u, ref)
    api.clear_workspace_cache()


def test_cloud100k_energy_records_on_the_default_stage(api, oracle):
    """md_run of the headline system (N = 1e5) on the default launch with an
    energy record every step: the recording steps take the row-group tiles
    with the pair energies.  The first record (the start state) and the last
    (the state the run ends in) against the oracle's kinetic, Coulomb and
    trap energies of those same states."""
    from _gpu_util import dev, state_host, state_tensors
    d = inputs.cloud100k()
    assert api.get_config("md_run", d["n"], "fp64")["algo"] == 4
    st = inputs.state9(d)
    ts = state_tensors(st)
    nsteps = 2
    en = api.md_run(ts, dev(d["q"]), dev(d["m"]), d["trap"], 0.0, d["dt"], nsteps, every=1).cpu().numpy()[0]
    got = state_host(ts)
    assert en.shape[0] == nsteps + 1 and api.poll_flags() == 0
    for rec, s in ((0, st), (nsteps, got)):
        t = rec * d["dt"]
        k = oracle.kinetic_energy(s[3], s[4], s[5], d["m"])
        u, _ = oracle.coulomb_energy(s[0], s[1], s[2], d["q"])
        tr = oracle.trap_energy(s[0], s[1], s[2], d["m"], d["trap"], t)
        ref = np.array([k, u, tr, k + u + tr])
        err = np.abs(en[rec] - ref)
        rel = np.divide(err, np.abs(ref), out=np.zeros(4), where=ref != 0)
        print(f"[cloud100k records] step {rec}: (K, U_C, U_trap, E) = {ref}, rel err {rel}", flush=True)
        assert np.all(err <= 1e-12 * np.abs(ref)), (rec, en[rec], ref)  # exact where ref is 0 (K at rest)
