"""GPU parity of coulomb_forces / coulomb_energy against the FP64 oracle
(called through the C ABI via the Python binding)."""
import numpy as np
import pytest

from paper_2106_11143_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_11143_amd import api as A
    A.lib()
    return A


def _forces(api, d, prec, eps2=0.0):
    from _gpu_util import dev, host
    f = api.coulomb_forces(dev(d["x"]), dev(d["y"]), dev(d["z"]), dev(d["q"]), eps2=eps2, prec=prec)
    return np.stack([host(t) for t in f])


@pytest.mark.parametrize("prec", ["fp64", "ieee", "mixed", "fp32"])
def test_forces_cloud1024_all_precisions(api, oracle, prec):
    from _gpu_util import PREC_TOL, per_ion_rel, report
    d = inputs.cloud1024()
    fx, fy, fz, kappa = oracle.forces(d["x"], d["y"], d["z"], d["q"], kappa=True)
    ref = np.stack([fx, fy, fz])
    F = _forces(api, d, prec)
    err = per_ion_rel(F, ref)
    report(f"cloud1024/{prec}", err, kappa)
    if prec == "fp32":
        assert np.all(err <= 2e-6 * np.maximum(kappa, 1.0))
    else:
        assert err.max() <= PREC_TOL[prec]
    assert api.poll_flags() == 0


RAGGED = [1, 2, 3, 7, 63, 64, 65, 127, 129, 255, 257, 1000, 1023, 1025, 2049]
CONFIGS = [(1, 64, 1), (1, 256, 3), (2, 128, 64), (4, 256, 5), (4, 64, 64), (2, 256, 1)]


@pytest.mark.parametrize("p,wg,splits", CONFIGS)
def test_forces_ragged_sizes_and_launch_shapes(api, oracle, p, wg, splits):
    from _gpu_util import per_ion_rel
    for n in RAGGED:
        g = np.random.Generator(np.random.PCG64(1000 + n))
        d = dict(x=g.normal(0, 20e-6, n), y=g.normal(0, 20e-6, n), z=g.normal(0, 20e-6, n),
                 q=inputs.E_CHARGE * g.choice([1.0, 2.0, -1.0], n))
        for prec in ("fp64", "mixed"):
            api.set_config("forces", n, prec, p=p, wg=wg, splits=splits)
            F = _forces(api, d, prec, eps2=(1e-7) ** 2 if n % 2 else 0.0)
            ref = np.stack(oracle.forces(d["x"], d["y"], d["z"], d["q"], eps2=(1e-7) ** 2 if n % 2 else 0.0))
            if n == 1:
                assert np.all(F == 0.0)
                continue
            err = per_ion_rel(F, ref)
            tol = 1e-12 if prec == "fp64" else 1e-7
            assert err.max() <= tol, (n, prec, err.max())
            api.reset_config("forces", n, prec)
    api.clear_workspace_cache()


SYM_SIZES = [1, 2, 3, 65, 127, 128, 129, 191, 192, 193, 320, 385, 511, 512, 513, 1000, 1537, 2049, 4001]
SYM_CONFIGS = [(1, 2, 256), (1, 3, 1024), (1, 4, 512), (1, 5, 2048), (1, 6, 256), (1, 8, 512),
               (2, 2, 512), (2, 4, 256), (2, 6, 1024), (2, 8, 512),
               (4, 4, 256), (4, 6, 512), (4, 8, 512), (4, 8, 2048), (4, 4, 1024)]


@pytest.mark.parametrize("algo,p,jl", SYM_CONFIGS)
def test_forces_symmetric_kernel_ragged_sizes(api, oracle, algo, p, jl):
    """The Newton's-third-law kernel (algo 1: reactions summed over the wave by
    permutes and DPP; algo 2: through LDS; algo 4: as 2 with four i-blocks per
    workgroup sharing each j-segment, their reactions added in LDS): i-blocks
    of 64p, j-segments of jl, ragged last blocks and segments, row groups with
    rows that have no pairs, sizes with no off-diagonal tile."""
    group = 4
    from _gpu_util import per_ion_rel
    for n in SYM_SIZES:
        g = np.random.Generator(np.random.PCG64(2000 + n))
        d = dict(x=g.normal(0, 20e-6, n), y=g.normal(0, 20e-6, n), z=g.normal(0, 20e-6, n),
                 q=inputs.E_CHARGE * g.choice([1.0, 2.0, -1.0], n))
        eps2 = (1e-7) ** 2 if n % 3 == 0 else 0.0
        ref = np.stack(oracle.forces(d["x"], d["y"], d["z"], d["q"], eps2=eps2))
        for prec in ("fp64", "mixed"):
            api.set_config("forces", n, prec, p=p, wg=group, splits=jl, algo=algo)
            F = _forces(api, d, prec, eps2=eps2)
            api.reset_config("forces", n, prec)
            if n == 1:
                assert np.all(F == 0.0)
                continue
            err = per_ion_rel(F, ref)
            assert err.max() <= (1e-12 if prec == "fp64" else 1e-7), (n, prec, p, jl, err.max())
            # each pair is applied to both ions: Newton's third law holds to rounding
            assert np.linalg.norm(F.sum(axis=1)) <= 1e-13 * np.linalg.norm(F, axis=0).sum()


def test_forces_rf32768_full(api, oracle):
    from _gpu_util import per_ion_rel, report
    d = inputs.rf32768()
    fx, fy, fz, kappa = oracle.forces(d["x"], d["y"], d["z"], d["q"], kappa=True)
    ref = np.stack([fx, fy, fz])
    for prec in ("fp64", "mixed"):
        F = _forces(api, d, prec)
        err = per_ion_rel(F, ref)
        report(f"rf32768/{prec}", err, kappa)
        assert err.max() <= (1e-12 if prec == "fp64" else 1e-7)


def test_forces_cloud100k_sampled(api, oracle):
    """Full-size workload in the default launch configuration: every GPU force
    is computed, a sample of ions is checked against the oracle one by one,
    and Newton's third law is checked on the whole result."""
    from _gpu_util import per_ion_rel, report
    d = inputs.cloud100k()
    n = d["n"]
    g = np.random.Generator(np.random.PCG64(77))
    idx = np.unique(np.concatenate([np.arange(64), np.arange(n - 64, n), g.choice(n, 1500, replace=False),
                                    np.flatnonzero(d["q"] > 1.5 * inputs.E_CHARGE)[:200]]))
    fx, fy, fz, kappa = oracle.forces(d["x"], d["y"], d["z"], d["q"], idx=idx, kappa=True)
    ref = np.stack([fx, fy, fz])
    for prec in ("fp64", "mixed"):
        F = _forces(api, d, prec)
        err = per_ion_rel(F[:, idx], ref)
        report(f"cloud100k/{prec} ({len(idx)} sampled)", err, kappa)
        assert err.max() <= (1e-12 if prec == "fp64" else 1e-7)
        tot = np.linalg.norm(F.sum(axis=1))
        assert tot <= 1e-12 * np.linalg.norm(F, axis=0).sum()


@pytest.mark.parametrize("n,i0,i1", [(1, 0, 1), (2, 1, 2), (4001, 0, 1), (4001, 37, 1000), (4001, 3900, 4001),
                                     (4001, 0, 4001), (300, 64, 129)])
def test_forces_range_ragged(api, oracle, n, i0, i1):
    """coulomb_forces_range: the forces on ions i0 .. i1-1 from all n ions,
    against the oracle on the same ions; ragged ranges, ranges that start
    inside a wave, the whole range."""
    from _gpu_util import dev, host, per_ion_rel
    g = np.random.Generator(np.random.PCG64(3000 + n + i0))
    d = dict(x=g.normal(0, 20e-6, n), y=g.normal(0, 20e-6, n), z=g.normal(0, 20e-6, n),
             q=inputs.E_CHARGE * g.choice([1.0, 2.0, -1.0], n))
    eps2 = (1e-7) ** 2 if i0 % 2 else 0.0
    idx = np.arange(i0, i1)
    ref = np.stack(oracle.forces(d["x"], d["y"], d["z"], d["q"], eps2=eps2, idx=idx))
    for prec in ("fp64", "mixed"):
        F = np.stack([host(t) for t in api.coulomb_forces_range(*(dev(d[k]) for k in "xyzq"), i0, i1, eps2=eps2,
                                                                 prec=prec)])
        assert F.shape == (3, i1 - i0)
        if n == 1:
            assert np.all(F == 0.0)
            continue
        err = per_ion_rel(F, ref)
        assert err.max() <= (1e-12 if prec == "fp64" else 1e-7), (n, i0, i1, prec, err.max())


def test_forces_range_one_gpu_share_of_cloud100k(api, oracle):
    """One GPU's share when N = 1e5 is split by ion index over 8 GPUs: ions
    37500 .. 49999 against all 1e5, sampled against the oracle."""
    from _gpu_util import dev, host, per_ion_rel, report
    d = inputs.cloud100k()
    n = d["n"]
    i0, i1 = 3 * n // 8, 4 * n // 8
    F = np.stack([host(t) for t in api.coulomb_forces_range(*(dev(d[k]) for k in "xyzq"), i0, i1)])
    g = np.random.Generator(np.random.PCG64(78))
    rel = np.unique(np.concatenate([[0, 1, i1 - i0 - 1], g.choice(i1 - i0, 400, replace=False)]))
    fx, fy, fz, kappa = oracle.forces(d["x"], d["y"], d["z"], d["q"], idx=i0 + rel, kappa=True)
    err = per_ion_rel(F[:, rel], np.stack([fx, fy, fz]))
    report("cloud100k share 3/8 (sampled)", err, kappa)
    assert err.max() <= 1e-12


@pytest.mark.parametrize("n", [1 << 18, (1 << 18) + 1])
def test_forces_at_the_symmetric_size_limit(api, oracle, n):
    """The largest size the Newton's-third-law stage takes (2^18 ions, its
    most tiles) and one more ion (the direct kernel takes over): sampled ions
    against the oracle."""
    from _gpu_util import dev, host, per_ion_rel, report
    d = inputs.cloud100k(n=n, seed=31)
    cfg = api.get_config("forces", n, "fp64")
    assert cfg["algo"] == (4 if n <= (1 << 18) else 0)  # row-group tiles up to 2^18
    F = np.stack([host(t) for t in api.coulomb_forces(*(dev(d[k]) for k in "xyzq"))])
    g = np.random.Generator(np.random.PCG64(79))
    idx = np.unique(np.concatenate([[0, 1, n - 2, n - 1], g.choice(n, 300, replace=False)]))
    fx, fy, fz, kappa = oracle.forces(d["x"], d["y"], d["z"], d["q"], idx=idx, kappa=True)
    err = per_ion_rel(F[:, idx], np.stack([fx, fy, fz]))
    report(f"n={n} algo={cfg['algo']} (sampled)", err, kappa)
    assert err.max() <= 1e-12
    api.clear_workspace_cache()


def test_fp32_displacement_ablation_error(api, oracle):
    """CB_MIXED_F32D, the literal "FP32 displacement" reading of the mixed
    path (displacements rounded to FP32 in r^2 and in the numerator), on the
    cloud100k shape at N = 6000: its error is reported, stays at the 2^-24
    level, and is far above CB_MIXED's (which keeps FP64 displacements)."""
    from _gpu_util import per_ion_rel, report
    d = inputs.cloud100k(n=6000, seed=12)
    fx, fy, fz, kappa = oracle.forces(d["x"], d["y"], d["z"], d["q"], kappa=True)
    ref = np.stack([fx, fy, fz])
    e_abl = per_ion_rel(_forces(api, d, "mixed_f32d"), ref)
    e_mix = per_ion_rel(_forces(api, d, "mixed"), ref)
    report("ablation fp32 displacement", e_abl, kappa)
    report("mixed (fp64 displacement)", e_mix, kappa)
    assert e_abl.max() < 1e-4 and np.sqrt(np.mean(e_abl ** 2)) < 1e-6
    assert e_abl.max() > 100 * e_mix.max()


def test_forces_are_deterministic(api):
    from _gpu_util import dev
    d = inputs.cloud1024(n=5000, seed=5)
    args = [dev(d[k]) for k in ("x", "y", "z", "q")]
    a = [t.clone() for t in api.coulomb_forces(*args)]
    b = api.coulomb_forces(*args)
    for u, v in zip(a, b):
        assert bool((u == v).all())


@pytest.mark.parametrize("n", [2, 1024, 32768])
def test_energy_parity(api, oracle, n):
    from _gpu_util import dev
    d = inputs.rf32768(n=n) if n > 1024 else inputs.cloud1024(n=n)
    ref, _ = oracle.coulomb_energy(d["x"], d["y"], d["z"], d["q"])
    for prec in ("fp64", "ieee", "mixed"):
        u = float(api.coulomb_energy(dev(d["x"]), dev(d["y"]), dev(d["z"]), dev(d["q"]), prec=prec)[0])
        tol = 1e-12 if prec != "mixed" else 1e-9
        assert abs(u - ref) <= tol * abs(ref), (prec, u, ref)


def test_nonfinite_flag_on_coincident_ions(api):
    from _gpu_util import dev
    x = np.array([0.0, 1e-6, 1e-6, 3e-6])
    z = np.zeros(4)
    q = np.full(4, inputs.E_CHARGE)
    api.poll_flags()
    f = api.coulomb_forces(dev(x), dev(z), dev(z), dev(q))
    assert api.poll_flags() & 1
    assert api.poll_flags() == 0  # cleared by the poll
    # softening makes the same configuration finite
    f = api.coulomb_forces(dev(x), dev(z), dev(z), dev(q), eps2=1e-14)
    assert api.poll_flags() == 0
    assert np.isfinite(np.stack([t.cpu().numpy() for t in f])).all()


@pytest.mark.parametrize("algo,p,jl", [(2, 2, 256), (2, 4, 512), (2, 8, 512), (2, 6, 1024), (4, 4, 256),
                                       (4, 8, 512)])
def test_energy_on_the_symmetric_stage(api, oracle, algo, p, jl):
    """coulomb_energy on the Newton's-third-law tiles (the potential summed
    as a fourth component, its reactions with the same sign): ragged sizes,
    mixed charges and ions grouped by species, against the oracle."""
    from _gpu_util import dev
    for k, n in enumerate([2, 3, 129, 513, 1000, 2049, 4001]):
        g = np.random.Generator(np.random.PCG64(9100 + n))
        d = dict(x=g.normal(0, 20e-6, n), y=g.normal(0, 20e-6, n), z=g.normal(0, 60e-6, n))
        if k % 2:
            d["q"] = inputs.E_CHARGE * g.choice([1.0, 2.0, -1.0], n)
        else:
            d["q"] = np.full(n, inputs.E_CHARGE)
            d["q"][int(0.7 * n):] = 2.0 * inputs.E_CHARGE
        eps2 = (1e-7) ** 2 if n % 2 else 0.0
        ref, _ = oracle.coulomb_energy(d["x"], d["y"], d["z"], d["q"], eps2=eps2)
        for prec, tol in (("fp64", 1e-12), ("mixed", 1e-9)):
            api.set_config("energy", n, prec, p=p, wg=4, splits=jl, algo=algo)
            try:
                u = float(api.coulomb_energy(*(dev(d[c]) for c in "xyzq"), eps2=eps2, prec=prec)[0])
            finally:
                api.reset_config("energy", n, prec)
            assert abs(u - ref) <= tol * abs(ref), (algo, p, jl, n, prec, u, ref)
    api.clear_workspace_cache()


def test_energy_records_on_the_symmetric_stage(api, oracle):
    """md_run at 20000 ions with an energy record every step: the recording
    steps take the Newton's-third-law stage with the potential (no direct
    fallback), records and state against the oracle's envelope; and
    coulomb_trap_grad's energy on the same stage."""
    from _gpu_util import dev, state_host, state_tensors
    n = 20000
    d = inputs.cloud1024(n=n, seed=21)
    st = inputs.state9(d)
    assert api.get_config("md_run", n, "fp64")["algo"] == 2
    nsteps = 4
    ref, en_ref, _ = oracle.md_run(st, d["q"], d["m"], d["trap"], 0.0, d["dt"], nsteps, every=1)
    perm = np.arange(n)[::-1]
    alt, en_alt, _ = oracle.md_run(st[:, perm], d["q"][perm], d["m"][perm], d["trap"], 0.0, d["dt"], nsteps, every=1)
    alt = alt[:, np.argsort(perm)]
    ts = state_tensors(st)
    en = api.md_run(ts, dev(d["q"]), dev(d["m"]), d["trap"], 0.0, d["dt"], nsteps, every=1)
    got = state_host(ts)
    for blk in (slice(0, 3), slice(3, 6), slice(6, 9)):
        D = np.abs(alt[blk] - ref[blk]).max()
        assert np.abs(got[blk] - ref[blk]).max() <= 10 * D + 1e-13 * np.abs(ref[blk]).max(), blk
    en = en.cpu().numpy()[0]
    print(f"[records n={n}] max energy err {np.abs(en - en_ref).max(axis=0)}", flush=True)
    assert np.all(np.abs(en - en_ref) <= 10 * np.abs(en_alt - en_ref) + 1e-12 * np.abs(en_ref).max(axis=0))
    # the gradient's energy (U_C + U_trap) on the same stage
    _, u = api.coulomb_trap_grad(*(dev(d[c]) for c in "xyzq"), dev(d["m"]), d["trap"], 0.0, energy=True)
    uref = oracle.coulomb_energy(d["x"], d["y"], d["z"], d["q"])[0] + \
        oracle.trap_energy(d["x"], d["y"], d["z"], d["m"], d["trap"], 0.0)
    assert abs(float(u[0]) - uref) <= 1e-12 * abs(uref)
