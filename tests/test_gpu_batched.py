"""GPU md_run with many runs of uneven size, on both ensemble paths (the
persistent kernel, one workgroup per run; the stepped path, two launches per
step over every run's Newton's-third-law tiles), against the oracle run by
run, against the single-run path and against each other."""
import contextlib

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


PERSISTENT = ("persistent",)
STEPPED4 = ("stepped", 4, 256)
STEPPED8 = ("stepped", 8, 512)
PATHS = [PERSISTENT, STEPPED4, STEPPED8]


@contextlib.contextmanager
def _path(api, ntot, prec, path):
    """Forces the ensemble path of md_run for ntot ions at prec."""
    if path[0] == "persistent":
        api.set_config("md_ensemble", ntot, prec, p=4, wg=512, splits=1, algo=0)
    else:
        api.set_config("md_ensemble", ntot, prec, p=path[1], wg=4, splits=path[2], algo=2)
    try:
        yield
    finally:
        api.reset_config("md_ensemble", ntot, prec)


def _ensemble(sizes, seed, trap):
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for n in sizes:
        sig = inputs.crystal_sigma(n, trap["wx"], trap["wy"], trap["wz"])
        pos = g.normal(size=(3, n)) * sig[:, None]
        vel = inputs.maxwell(g, n, 10e-3, inputs.MASS_40U)
        st = np.zeros((9, n))
        st[:3], st[3:6] = pos, vel
        parts.append(st)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    q = np.full(offs[-1], inputs.E_CHARGE)
    q[::7] *= 2.0
    m = np.full(offs[-1], inputs.MASS_40U)
    return parts, offs, q, m


def _check_run(oracle, st, q, m, trap, dt, nsteps, got, en_got, every, tag):
    ref, en, _ = oracle.md_run(st, q, m, trap, 0.0, dt, nsteps, every=every)
    perm = np.arange(len(q))[::-1]
    alt, en2, _ = oracle.md_run(st[:, perm], q[perm], m[perm], trap, 0.0, dt, nsteps, every=every)
    alt = alt[:, np.argsort(perm)]
    for blk in (slice(0, 3), slice(3, 6), slice(6, 9)):
        D = np.abs(alt[blk] - ref[blk]).max()
        err = np.abs(got[blk] - ref[blk]).max()
        assert err <= 10 * D + 1e-13 * np.abs(ref[blk]).max(), (tag, blk, err, D)
    if en_got is not None:
        assert np.all(np.abs(en_got - en) <= 10 * np.abs(en2 - en) + 1e-12 * np.abs(en).max(axis=0)), tag


@pytest.mark.parametrize("path", PATHS, ids=lambda p: "-".join(map(str, p)))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_ramp_matches_oracle_run_by_run(api, oracle, prec, path):
    from _gpu_util import dev
    trap = inputs.ramp_trap(1.5e6, 0.6e6, 0.15e6, 0.0, 60e-9)
    sizes = [64, 65, 130, 257, 500, 1000, 333]
    parts, offs, q, m = _ensemble(sizes, 3, trap)
    st = np.concatenate(parts, axis=1)
    ts = [dev(st[k]) for k in range(9)]
    dt, nsteps, every = 2e-9, 40, 10
    with _path(api, offs[-1], prec, path):
        en = api.md_run(ts, dev(q), dev(m), [trap] * len(sizes), 0.0, dt, nsteps, offsets=offs, every=every,
                        prec=prec)
    got = np.stack([t.cpu().numpy() for t in ts])
    en = en.cpu().numpy()
    for r, n in enumerate(sizes):
        sl = slice(offs[r], offs[r + 1])
        if prec == "fp64":
            _check_run(oracle, parts[r], q[sl], m[sl], trap, dt, nsteps, got[:, sl], en[r], every, f"run{r}")
        else:
            ref, _, _ = oracle.md_run(parts[r], q[sl], m[sl], trap, 0.0, dt, nsteps)
            assert np.abs(got[:3, sl] - ref[:3]).max() <= 1e-9 * np.abs(ref[:3]).max()
    assert api.poll_flags() == 0


@pytest.mark.parametrize("path", PATHS, ids=lambda p: "-".join(map(str, p)))
def test_batched_rf_drive_with_a_term_and_phase_matches_oracle(api, oracle, path):
    """Runs of one ensemble, each with its own RF drive with a DC term and a
    phase (a != 0, phi != 0), against the oracle run by run, on both ensemble
    paths."""
    from _gpu_util import dev
    sizes = [64, 300, 1000, 257]
    traps = [inputs.rf_trap(0.02, 0.3, 10e6, 0.15e6, phase=0.7), inputs.rf_trap(-0.03, 0.25, 10e6, 0.2e6, phase=2.5),
             inputs.rf_trap(0.01, 0.3, 8e6, 0.15e6, phase=-1.1), inputs.rf_trap(0.0, 0.2, 10e6, 0.1e6, phase=0.3)]
    parts, offs, q, m = _ensemble(sizes, 17, inputs.pseudo_trap(1.0e6, 1.0e6, 0.15e6))
    st = np.concatenate(parts, axis=1)
    ts = [dev(st[k]) for k in range(9)]
    dt, nsteps, every = 5e-9, 30, 10
    with _path(api, offs[-1], "fp64", path):
        en = api.md_run(ts, dev(q), dev(m), traps, 0.0, dt, nsteps, offsets=offs, every=every)
    got = np.stack([t.cpu().numpy() for t in ts])
    en = en.cpu().numpy()
    for r in range(len(sizes)):
        sl = slice(offs[r], offs[r + 1])
        _check_run(oracle, parts[r], q[sl], m[sl], traps[r], dt, nsteps, got[:, sl], en[r], every, f"run{r}")
    assert api.poll_flags() == 0


@pytest.mark.parametrize("path", PATHS, ids=lambda p: "-".join(map(str, p)))
def test_batched_equals_single_run_path(api, path):
    from _gpu_util import dev
    trap = inputs.pseudo_trap(1.0e6, 1.0e6, 0.15e6)
    sizes = [200, 96, 1500]
    parts, offs, q, m = _ensemble(sizes, 5, trap)
    st = np.concatenate(parts, axis=1)
    ts = [dev(st[k]) for k in range(9)]
    with _path(api, offs[-1], "fp64", path):
        api.md_run(ts, dev(q), dev(m), [trap] * 3, 0.0, 1e-9, 25, offsets=offs)
    got = np.stack([t.cpu().numpy() for t in ts])
    for r in range(3):
        sl = slice(offs[r], offs[r + 1])
        one = [dev(parts[r][k]) for k in range(9)]
        api.md_run(one, dev(q[sl]), dev(m[sl]), trap, 0.0, 1e-9, 25)
        single = np.stack([t.cpu().numpy() for t in one])
        for blk in (slice(0, 3), slice(3, 6)):
            scale = np.abs(single[blk]).max()
            assert np.abs(got[blk, sl] - single[blk]).max() <= 1e-11 * scale


@pytest.mark.parametrize("path", PATHS, ids=lambda p: "-".join(map(str, p)))
def test_batched_largest_run_and_order(api, oracle, path):
    """A 4096-ion run (the size limit) mixed with small ones; the persistent
    kernel takes runs largest first and the stepped path launches tiles
    longest first, but each run lands in its own slice."""
    from _gpu_util import dev
    trap = inputs.pseudo_trap(1.0e6, 1.0e6, 0.15e6)
    sizes = [70, 4096, 64, 2049]
    parts, offs, q, m = _ensemble(sizes, 8, trap)
    st = np.concatenate(parts, axis=1)
    ts = [dev(st[k]) for k in range(9)]
    with _path(api, offs[-1], "fp64", path):
        api.md_run(ts, dev(q), dev(m), [trap] * 4, 0.0, 1e-9, 3, offsets=offs)
    got = np.stack([t.cpu().numpy() for t in ts])
    for r in (0, 1, 3):
        sl = slice(offs[r], offs[r + 1])
        _check_run(oracle, parts[r], q[sl], m[sl], trap, 1e-9, 3, got[:, sl], None, 1, f"run{r}")


def test_kz_ensemble_small(api):
    """The Kibble-Zurek workload at reduced size: 24 runs, N in [64, 600],
    the ramp, 300 steps, energies recorded; defect counts are reported
    (operational definition, not pinned)."""
    import torch
    from paper_2106_11143_amd import drivers
    from _gpu_util import dev
    d = inputs.kz512(nrun=24, nmin=64, nmax=600, nsteps=300)
    st = inputs.state9(d)
    ts = [dev(st[k]) for k in range(9)]
    en = api.md_run(ts, dev(d["q"]), dev(d["m"]), d["traps"], 0.0, d["dt"], d["nsteps"], offsets=d["offsets"],
                    every=100)
    assert api.poll_flags() == 0
    got = np.stack([t.cpu().numpy() for t in ts])
    assert np.isfinite(got).all() and np.isfinite(en.cpu().numpy()).all()
    offs = d["offsets"]
    counts = [drivers.count_defects(got[0, offs[r]:offs[r + 1]], got[1, offs[r]:offs[r + 1]],
                                    got[2, offs[r]:offs[r + 1]]) for r in range(24)]
    print(f"[kz small] defect counts {counts}", flush=True)


@pytest.mark.parametrize("path", PATHS, ids=lambda p: "-".join(map(str, p)))
def test_batched_with_friction_matches_oracle_run_by_run(api, oracle, path):
    """Runs with different friction coefficients (one of them zero) in one
    md_run, each against the oracle."""
    from _gpu_util import dev
    base = inputs.pseudo_trap(1.0e6, 1.0e6, 0.15e6)
    traps = [dict(base, gamma=g * inputs.MASS_40U) for g in (0.0, 2e5, 1e6)]
    sizes = [130, 64, 600]
    parts, offs, q, m = _ensemble(sizes, 17, base)
    st = np.concatenate(parts, axis=1)
    ts = [dev(st[k]) for k in range(9)]
    nsteps, every = 40, 10
    with _path(api, offs[-1], "fp64", path):
        en = api.md_run(ts, dev(q), dev(m), traps, 0.0, 2e-9, nsteps, offsets=offs, every=every).cpu().numpy()
    got = np.stack([t.cpu().numpy() for t in ts])
    for r in range(3):
        sl = slice(offs[r], offs[r + 1])
        _check_run(oracle, parts[r], q[sl], m[sl], traps[r], 2e-9, nsteps, got[:, sl], en[r], every, f"run {r}")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_newton_pass_matches_oracle(api, oracle, prec):
    """In the persistent kernel, runs above 3072 ions take the Newton's-third-law block-pair pass
    (round-robin over 256-ion blocks, ragged last block); a small run in the
    same launch takes the direct pass.  Each run against the oracle, with
    energies recorded every 4 steps (recording steps use the direct pass)."""
    from _gpu_util import dev
    trap = inputs.pseudo_trap(1.0e6, 1.0e6, 0.15e6)
    sizes = [3073, 4096, 3500, 130]
    parts, offs, q, m = _ensemble(sizes, 23, trap)
    st = np.concatenate(parts, axis=1)
    ts = [dev(st[k]) for k in range(9)]
    nsteps, every = 10, 4
    with _path(api, offs[-1], prec, PERSISTENT):
        en = api.md_run(ts, dev(q), dev(m), [trap] * len(sizes), 0.0, 2e-9, nsteps, offsets=offs, every=every,
                        prec=prec).cpu().numpy()
    got = np.stack([t.cpu().numpy() for t in ts])
    for r in range(len(sizes)):
        sl = slice(offs[r], offs[r + 1])
        _check_run(oracle, parts[r], q[sl], m[sl], trap, 2e-9, nsteps, got[:, sl], en[r], every, f"run {r}")
    assert api.poll_flags() == 0


@pytest.mark.parametrize("path", [STEPPED4, STEPPED8], ids=lambda p: "-".join(map(str, p)))
@pytest.mark.parametrize("prec", ["fp64", "ieee"])
def test_stepped_ensemble_block_edges_and_traps(api, oracle, prec, path):
    """The stepped path on run sizes at and around its i-block (64 p) and
    segment edges, a single-ion run, and one trap kind per run (static,
    ramp, RF drive, friction), energies every step; each run against the
    oracle."""
    from _gpu_util import dev
    base = inputs.pseudo_trap(1.0e6, 1.0e6, 0.15e6)
    kinds = [base, inputs.ramp_trap(1.5e6, 0.6e6, 0.15e6, 0.0, 20e-9),
             inputs.rf_trap(0.0, 0.3, 10e6, 0.15e6), dict(base, gamma=5e5 * inputs.MASS_40U)]
    sizes = [1, 63, 64, 65, 255, 256, 257, 511, 512, 513, 769, 1100, 1537]
    traps = [kinds[r % 4] for r in range(len(sizes))]
    parts, offs, q, m = _ensemble(sizes, 29, base)
    st = np.concatenate(parts, axis=1)
    ts = [dev(st[k]) for k in range(9)]
    nsteps, every = 12, 1
    with _path(api, offs[-1], prec, path):
        en = api.md_run(ts, dev(q), dev(m), traps, 0.0, 1e-9, nsteps, offsets=offs, every=every,
                        prec=prec).cpu().numpy()
    got = np.stack([t.cpu().numpy() for t in ts])
    for r, n in enumerate(sizes):
        sl = slice(offs[r], offs[r + 1])
        if n == 1:  # no pairs: the trap alone, against the oracle's trajectory
            ref, en_ref, _ = oracle.md_run(parts[r], q[sl], m[sl], traps[r], 0.0, 1e-9, nsteps, every=every)
            assert np.abs(got[:, sl] - ref).max() <= 1e-12 * np.abs(ref).max()
            assert np.abs(en[r] - en_ref).max() <= 1e-12 * np.abs(en_ref).max()
            continue
        _check_run(oracle, parts[r], q[sl], m[sl], traps[r], 1e-9, nsteps, got[:, sl], en[r], every, f"run {r} n={n}")
    assert api.poll_flags() == 0


@pytest.mark.parametrize("path,nrun", [(STEPPED4, 40), (STEPPED8, 40), (STEPPED4, 120)],
                         ids=["stepped-4-256-40", "stepped-8-512-40", "stepped-4-256-120"])
def test_stepped_equals_persistent_and_is_deterministic(api, path, nrun):
    """A Kibble-Zurek-shaped ensemble (N uniform in [64, 4096], the ramp) on
    both paths: trajectories agree to rounding (different summation orders),
    and the stepped path repeats bit for bit.  Also without CB_INIT_ACCEL
    (the state's a is used as a_0).  40 runs make a launch of fewer than
    4096 off-diagonal tiles (each block's diagonal split into sub-tiles of
    128 j's); 120 runs at 256-ion blocks make more (whole diagonals) and
    more than 4096 64-ion chunks (2 finishing waves per chunk, not 4)."""
    import torch
    from _gpu_util import dev
    d = inputs.kz512(nrun=nrun, nmin=64, nmax=4096, nsteps=6)
    st = inputs.state9(d)
    q, m, offs = dev(d["q"]), dev(d["m"]), d["offsets"]
    runs = {}
    for tag, pth, init in (("persistent", PERSISTENT, True), ("stepped", path, True), ("again", path, True),
                           ("persistent_a0", PERSISTENT, False), ("stepped_a0", path, False)):
        ts = [dev(st[k]) for k in range(9)]
        if not init:  # a_0 from one force evaluation of the start state (same on both paths)
            a0 = [dev(st[k]) for k in range(9)]
            with _path(api, offs[-1], "fp64", PERSISTENT):
                api.md_run(a0, q, m, d["traps"], 0.0, d["dt"], 0, offsets=offs)
            for k in range(6, 9):
                ts[k].copy_(a0[k])
        with _path(api, offs[-1], "fp64", pth):
            en = api.md_run(ts, q, m, d["traps"], 0.0, d["dt"], d["nsteps"], offsets=offs, every=3,
                            init_accel=init)
        torch.cuda.synchronize()
        runs[tag] = (np.stack([t.cpu().numpy() for t in ts]), en.cpu().numpy())
    assert api.poll_flags() == 0
    assert np.array_equal(runs["stepped"][0], runs["again"][0])
    assert np.array_equal(runs["stepped"][1], runs["again"][1])
    for a, b in (("persistent", "stepped"), ("persistent_a0", "stepped_a0")):
        ga, gb = runs[a][0], runs[b][0]
        for blk in (slice(0, 3), slice(3, 6), slice(6, 9)):
            scale = np.abs(ga[blk]).max()
            err = np.abs(ga[blk] - gb[blk]).max()
            print(f"[{a} vs {b}] block {blk.start}: max diff {err / scale:.2e} of scale", flush=True)
            assert err <= 1e-11 * scale, (a, b, blk, err / scale)
        ea, eb = runs[a][1], runs[b][1]
        assert np.abs(ea - eb).max() <= 1e-11 * np.abs(ea).max()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_stepped_whole_run_blocks_match_oracle(api, oracle, prec):
    """Every run within one 512-ion i-block (the default shape when no run
    exceeds 512 ions): no pair launch, the step kernel evaluates each run's
    pairs directly with 16 waves per 64 ions.  Sizes from 1 to 512, every
    trap kind and friction, energies every other step, against the oracle
    run by run and against the persistent kernel."""
    from _gpu_util import dev
    base = inputs.pseudo_trap(1.0e6, 1.0e6, 0.15e6)
    kinds = [base, inputs.ramp_trap(1.5e6, 0.6e6, 0.15e6, 0.0, 20e-9),
             inputs.rf_trap(0.0, 0.3, 10e6, 0.15e6), dict(base, gamma=5e5 * inputs.MASS_40U)]
    sizes = [1, 5, 64, 100, 257, 512, 333, 65]
    traps = [kinds[r % 4] for r in range(len(sizes))]
    parts, offs, q, m = _ensemble(sizes, 31, base)
    st = np.concatenate(parts, axis=1)
    nsteps, every = 10, 2
    got = {}
    for path in (STEPPED8, PERSISTENT):
        ts = [dev(st[k]) for k in range(9)]
        with _path(api, offs[-1], prec, path):
            en = api.md_run(ts, dev(q), dev(m), traps, 0.0, 1e-9, nsteps, offsets=offs, every=every,
                            prec=prec).cpu().numpy()
        got[path] = (np.stack([t.cpu().numpy() for t in ts]), en)
    assert api.poll_flags() == 0
    a, b = got[STEPPED8], got[PERSISTENT]
    for blk in (slice(0, 3), slice(3, 6), slice(6, 9)):
        assert np.abs(a[0][blk] - b[0][blk]).max() <= 1e-11 * np.abs(b[0][blk]).max()
    assert np.abs(a[1] - b[1]).max() <= 1e-11 * np.abs(b[1]).max()
    if prec == "fp64":
        for r, n in enumerate(sizes):
            sl = slice(offs[r], offs[r + 1])
            if n == 1:
                ref, en_ref, _ = oracle.md_run(parts[r], q[sl], m[sl], traps[r], 0.0, 1e-9, nsteps, every=every)
                assert np.abs(a[0][:, sl] - ref).max() <= 1e-12 * np.abs(ref).max()
                assert np.abs(a[1][r] - en_ref).max() <= 1e-12 * np.abs(en_ref).max()
                continue
            _check_run(oracle, parts[r], q[sl], m[sl], traps[r], 1e-9, nsteps, a[0][:, sl], a[1][r], every,
                       f"run {r} n={n}")


@pytest.mark.parametrize("path", [STEPPED4, PERSISTENT], ids=lambda p: "-".join(map(str, p)))
def test_ensemble_zero_steps_and_softening(api, oracle, path):
    """nsteps = 0 with CB_INIT_ACCEL and a record: the state is unchanged but
    for a_0, and the one record is the oracle's energy at t0; then a short
    run with softening eps2 > 0 against the oracle."""
    from _gpu_util import dev
    trap = inputs.pseudo_trap(1.0e6, 1.0e6, 0.15e6)
    sizes = [700, 64, 1300]
    parts, offs, q, m = _ensemble(sizes, 37, trap)
    st = np.concatenate(parts, axis=1)
    ts = [dev(st[k]) for k in range(9)]
    with _path(api, offs[-1], "fp64", path):
        en = api.md_run(ts, dev(q), dev(m), [trap] * 3, 0.0, 1e-9, 0, offsets=offs, every=1).cpu().numpy()
    got = np.stack([t.cpu().numpy() for t in ts])
    assert np.array_equal(got[:6], st[:6])
    for r in range(3):
        sl = slice(offs[r], offs[r + 1])
        ref, en_ref, _ = oracle.md_run(parts[r], q[sl], m[sl], trap, 0.0, 1e-9, 0, every=1)
        assert np.abs(got[6:, sl] - ref[6:]).max() <= 1e-12 * np.abs(ref[6:]).max()
        assert np.abs(en[r] - en_ref).max() <= 1e-12 * np.abs(en_ref).max()
    eps2 = (2e-6) ** 2
    ts = [dev(st[k]) for k in range(9)]
    with _path(api, offs[-1], "fp64", path):
        api.md_run(ts, dev(q), dev(m), [trap] * 3, 0.0, 1e-9, 5, offsets=offs, eps2=eps2)
    got = np.stack([t.cpu().numpy() for t in ts])
    for r in range(3):
        sl = slice(offs[r], offs[r + 1])
        ref, _, _ = oracle.md_run(parts[r], q[sl], m[sl], trap, 0.0, 1e-9, 5, eps2=eps2)
        for blk in (slice(0, 3), slice(3, 6), slice(6, 9)):
            assert np.abs(got[blk, sl] - ref[blk]).max() <= 1e-11 * np.abs(ref[blk]).max(), (r, blk)


@pytest.mark.parametrize("path,sizes", [(PERSISTENT, [100, 300, 700]), (STEPPED4, [100, 300, 700]),
                                        (STEPPED8, [100, 300, 700]), (STEPPED8, [100, 300, 500])],
                         ids=["persistent", "stepped-4-256", "stepped-8-512", "stepped-whole"])
def test_ensemble_captured_in_a_hip_graph_replays_bitwise(api, path, sizes):
    """md_run with several runs on a capturing stream: its run tables and
    traps go into host memory that the graph owns, so every replay equals
    the eager run bitwise (state and energy records), although the offsets
    and trap arrays of the captured call are gone and an eager call on other
    runs of the same total (other tables in the same workspace) runs
    between replays.  Both paths, the stepped one with tiles and with every
    run a single block."""
    import torch
    from _gpu_util import dev
    trap0 = inputs.pseudo_trap(1.0e6, 1.0e6, 0.15e6)
    traps = [inputs.pseudo_trap(1.0e6 * (1 + 0.1 * r), 1.0e6, 0.15e6 * (1 + 0.05 * r)) for r in range(len(sizes))]
    parts, offs, q, m = _ensemble(sizes, 43, trap0)
    st = np.concatenate(parts, axis=1)
    ntot = int(offs[-1])
    qd, md = dev(q), dev(m)
    nsteps, every, dt = 12, 3, 1e-9
    other_sizes = sizes[::-1]
    oparts, ooffs, _, _ = _ensemble(other_sizes, 44, trap0)
    ost = np.concatenate(oparts, axis=1)
    with _path(api, ntot, "fp64", path):
        eager = [dev(st[k]) for k in range(9)]
        en_eager = api.md_run(eager, qd, md, traps, 0.0, dt, nsteps, offsets=offs, every=every,
                              init_accel=True).clone()
        ref = torch.stack(eager)
        static = [dev(st[k]) for k in range(9)]
        api.md_run(static, qd, md, traps, 0.0, dt, 2, offsets=offs, every=every)  # warm-up: workspace
        torch.cuda.synchronize()
        s0 = torch.stack([dev(st[k]) for k in range(9)])
        for k in range(9):
            static[k].copy_(s0[k])
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            en_static = api.md_run(static, qd, md, [dict(t) for t in traps], 0.0, dt, nsteps,
                                   offsets=[int(o) for o in offs], every=every, init_accel=True)
        for rep in range(3):
            for k in range(9):
                static[k].copy_(s0[k])
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(torch.stack(static), ref), rep
            assert torch.equal(en_static, en_eager), rep
            other = [dev(ost[k]) for k in range(9)]  # other tables in the same workspace
            api.md_run(other, qd, md, trap0, 0.0, dt, 3, offsets=ooffs, init_accel=True)
            torch.cuda.synchronize()
            assert torch.isfinite(torch.stack(other)).all()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_kz512_full_ensemble_sampled_runs_match_oracle(api, oracle, prec):
    """The full Kibble-Zurek ensemble (512 runs, N uniform in [64, 4096],
    about 1.07e6 ions, the ramped trap) in the default launch that bench.py
    times: three steps with an energy record after each, then the largest
    and the smallest run and six seeded others against the oracle run by
    run, every ion of each.  FP64: positions, velocities, accelerations and
    energies within ten times the oracle's own round-off envelope; mixed:
    positions and velocities within 1e-9 of each block's scale."""
    from _gpu_util import dev
    d = inputs.kz512()
    offs = d["offsets"]
    sizes = np.diff(offs)
    st = inputs.state9(d)
    ts = [dev(st[k]) for k in range(9)]
    nsteps, every = 3, 1
    print(f"[kz512 full {prec}] {len(sizes)} runs, {int(offs[-1])} ions", flush=True)
    en = api.md_run(ts, dev(d["q"]), dev(d["m"]), d["traps"], 0.0, d["dt"], nsteps, offsets=offs, every=every,
                    prec=prec)
    assert api.poll_flags() == 0
    got = np.stack([t.cpu().numpy() for t in ts])
    en = en.cpu().numpy()
    assert np.isfinite(got).all() and np.isfinite(en).all()
    g = np.random.Generator(np.random.PCG64(512))
    runs = sorted({int(np.argmax(sizes)), int(np.argmin(sizes))} |
                  {int(r) for r in g.choice(len(sizes), 6, replace=False)})
    for r in runs:
        sl = slice(int(offs[r]), int(offs[r + 1]))
        tag = f"kz512 run {r} (N = {int(sizes[r])})"
        if prec == "fp64":
            _check_run(oracle, st[:, sl], d["q"][sl], d["m"][sl], d["traps"][r], d["dt"], nsteps, got[:, sl], en[r],
                       every, tag)
        else:
            ref, _, _ = oracle.md_run(st[:, sl], d["q"][sl], d["m"][sl], d["traps"][r], 0.0, d["dt"], nsteps)
            for blk in (slice(0, 3), slice(3, 6)):
                assert np.abs(got[blk, sl] - ref[blk]).max() <= 1e-9 * np.abs(ref[blk]).max(), (tag, blk)
    print(f"[kz512 full {prec}] runs {runs} match the oracle", flush=True)
