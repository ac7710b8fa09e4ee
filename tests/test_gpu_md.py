"""GPU velocity-Verlet (md_step / md_run, single run) against the oracle and
against closed forms."""
import math

import numpy as np
import pytest

from paper_2106_11143_amd import inputs

pytestmark = pytest.mark.gpu
E = inputs.E_CHARGE
M40 = inputs.MASS_40U


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_11143_amd import api as A
    A.lib()
    return A


def _oracle_envelope(oracle, st, q, m, trap, dt, nsteps, every):
    """Oracle run and its round-off envelope: the same run with the ions in
    reversed order (a different summation order)."""
    ref, en, _ = oracle.md_run(st, q, m, trap, 0.0, dt, nsteps, every=every)
    perm = np.arange(len(q))[::-1]
    alt, en2, _ = oracle.md_run(st[:, perm], q[perm], m[perm], trap, 0.0, dt, nsteps, every=every)
    inv = np.argsort(perm)
    return ref, en, alt[:, inv], en2


def test_md_run_cloud1024_matches_oracle(api, oracle):
    from _gpu_util import dev, state_host, state_tensors
    d = inputs.cloud1024()
    st = inputs.state9(d)
    dt, nsteps = d["dt"], d["nsteps"]
    ref, en_ref, alt, en_alt = _oracle_envelope(oracle, st, d["q"], d["m"], d["trap"], dt, nsteps, 1)
    ts = state_tensors(st)
    en = api.md_run(ts, dev(d["q"]), dev(d["m"]), d["trap"], 0.0, dt, nsteps, every=1)
    got = state_host(ts)
    for blk, scale in ((slice(0, 3), np.abs(ref[:3]).max()), (slice(3, 6), np.abs(ref[3:6]).max()),
                       (slice(6, 9), np.abs(ref[6:9]).max())):
        D = np.abs(alt[blk] - ref[blk]).max()
        err = np.abs(got[blk] - ref[blk]).max()
        print(f"[md cloud1024] block {blk}: err={err:.3e} envelope={D:.3e} scale={scale:.3e}", flush=True)
        assert err <= 10 * D + 1e-13 * scale
    en = en.cpu().numpy()[0]
    Escale = np.abs(en_ref).max(axis=0)
    dE = np.abs(en - en_ref).max(axis=0)
    env = np.abs(en_alt - en_ref).max(axis=0)
    print(f"[md cloud1024] energy err={dE} envelope={env}", flush=True)
    assert np.all(dE <= 10 * env + 1e-12 * Escale)
    assert api.poll_flags() == 0


def test_md_step_equals_one_step_run(api):
    from _gpu_util import dev, state_host, state_tensors
    d = inputs.cloud1024(n=777, seed=3)
    st = inputs.state9(d)
    a = state_tensors(st)
    q, m = dev(d["q"]), dev(d["m"])
    api.md_run(a, q, m, d["trap"], 0.0, 1e-9, 0, init_accel=True)  # a_0 only
    b = [t.clone() for t in a]
    api.md_step(a, q, m, d["trap"], 0.0, 1e-9)
    api.md_run(b, q, m, d["trap"], 0.0, 1e-9, 1, init_accel=False)
    assert np.array_equal(state_host(a), state_host(b))


def test_checkpoint_resume_is_bitwise(api):
    from _gpu_util import dev, state_host, state_tensors
    d = inputs.cloud1024(n=1500, seed=4)
    st = inputs.state9(d)
    q, m = dev(d["q"]), dev(d["m"])
    a = state_tensors(st)
    api.md_run(a, q, m, d["trap"], 0.0, 1e-9, 100)
    b = state_tensors(st)
    api.md_run(b, q, m, d["trap"], 0.0, 1e-9, 50)
    saved = state_host(b)
    c = state_tensors(saved)
    api.md_run(c, q, m, d["trap"], 50e-9, 1e-9, 50, init_accel=False)
    assert np.array_equal(state_host(a), state_host(c))


@pytest.mark.parametrize("n", [20000, 90000])
def test_checkpoint_resume_is_bitwise_on_the_symmetric_stage(api, n):
    """md_run on the Newton's-third-law stage (one wave per tile at 20000
    ions, row groups at 90000), energies every other step: the tile table is
    built by a run's first force stage and read by its later ones, so one
    6-step run and a 4-step run resumed for 2 steps (a new call, a new table)
    must agree bitwise, state and records."""
    from _gpu_util import dev, state_host, state_tensors
    d = inputs.cloud1024(n=n, seed=6)
    assert api.get_config("md_run", n, "fp64")["algo"] == (2 if n < 81920 else 4)
    st = inputs.state9(d)
    q, m = dev(d["q"]), dev(d["m"])
    a = state_tensors(st)
    ea = api.md_run(a, q, m, d["trap"], 0.0, 1e-9, 6, every=2)
    b = state_tensors(st)
    eb = api.md_run(b, q, m, d["trap"], 0.0, 1e-9, 4, every=2)
    c = state_tensors(state_host(b))
    ec = api.md_run(c, q, m, d["trap"], 4e-9, 1e-9, 2, every=2, init_accel=False)
    assert np.array_equal(state_host(a), state_host(c))
    ea, eb, ec = (e.cpu().numpy() for e in (ea, eb, ec))
    assert np.array_equal(ea[0, :3], eb[0])  # records of steps 0, 2, 4
    assert np.array_equal(eb[0, 2], ec[0, 0])  # step 4, recorded at the end of one call and the start of the next
    assert np.array_equal(ea[0, 3], ec[0, 1])  # step 6


@pytest.mark.parametrize("fz_hz", [0.2e6, 0.05e6])
def test_two_ion_crystal_stays_put(api, fz_hz):
    from _gpu_util import dev, state_host, state_tensors
    wz = 2 * math.pi * fz_hz
    d = (2.0 * 8.9875517923e9 * E * E / (M40 * wz * wz)) ** (1.0 / 3.0)
    st = np.zeros((9, 2))
    st[2] = [d / 2, -d / 2]
    ts = state_tensors(st)
    api.md_run(ts, dev([E, E]), dev([M40, M40]), inputs.pseudo_trap(1e6, 1e6, fz_hz), 0.0, 1e-9, 2000)
    out = state_host(ts)
    assert np.abs(out[2] - st[2]).max() <= 1e-9 * d
    assert np.abs(out[:2]).max() == 0.0


def test_single_ion_rf_matches_oracle(api, oracle):
    from _gpu_util import dev, state_host, state_tensors
    trap = inputs.rf_trap(0.0, 0.3, 10e6, 0.1e6)
    st = np.zeros((9, 1))
    st[:3, 0] = [1e-6, -2e-6, 0.5e-6]
    st[3:6, 0] = [0.3, 0.1, -0.2]
    dt = 5e-9
    ref, _, _ = oracle.md_run(st, [E], [M40], trap, 0.0, dt, 400)
    ts = state_tensors(st)
    api.md_run(ts, dev([E]), dev([M40]), trap, 0.0, dt, 400)
    got = state_host(ts)
    for blk in (slice(0, 3), slice(3, 6)):
        assert np.abs(got[blk] - ref[blk]).max() <= 1e-12 * np.abs(ref[blk]).max()


def test_rf32768_steps_match_oracle(api, oracle):
    from _gpu_util import dev, state_host, state_tensors
    d = inputs.rf32768()
    st = inputs.state9(d)
    nsteps = 6
    ref, en_ref, alt, en_alt = _oracle_envelope(oracle, st, d["q"], d["m"], d["trap"], d["dt"], nsteps, 3)
    ts = state_tensors(st)
    en = api.md_run(ts, dev(d["q"]), dev(d["m"]), d["trap"], 0.0, d["dt"], nsteps, every=3)
    got = state_host(ts)
    for blk in (slice(0, 3), slice(3, 6), slice(6, 9)):
        D = np.abs(alt[blk] - ref[blk]).max()
        err = np.abs(got[blk] - ref[blk]).max()
        assert err <= 10 * D + 1e-13 * np.abs(ref[blk]).max()
    en = en.cpu().numpy()[0]
    assert np.all(np.abs(en - en_ref) <= 10 * np.abs(en_alt - en_ref) + 1e-12 * np.abs(en_ref).max(axis=0))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cloud100k_centre_of_mass_follows_harmonic_solution(api, prec):
    """Kohn's theorem for the discrete run: the Coulomb forces sum to zero, so
    in a static harmonic trap the centre of mass of equal-mass ions follows
    the single-ion velocity-Verlet solution exactly, at any N."""
    from _gpu_util import dev, state_host, state_tensors
    d = inputs.cloud100k()
    st = inputs.state9(d)
    nsteps, dt = d["nsteps"], d["dt"]
    ts = state_tensors(st)
    api.md_run(ts, dev(d["q"]), dev(d["m"]), d["trap"], 0.0, dt, nsteps, prec=prec)
    out = state_host(ts)
    n = np.arange(nsteps + 1)
    for c, w in enumerate((d["trap"]["wx"], d["trap"]["wy"], d["trap"]["wz"])):
        th = 2.0 * math.asin(w * dt / 2.0)
        A = st[c].mean()
        com = A * math.cos(nsteps * th)
        spread = np.abs(out[c]).max()
        assert abs(out[c].mean() - com) <= 1e-11 * spread, (c, out[c].mean(), com)
    assert api.poll_flags() == 0


@pytest.mark.parametrize("n,every", [(1024, 1), (20000, 10)])
def test_md_run_with_friction_matches_oracle(api, oracle, n, every):
    """eq. (1)'s friction term (trapezoidal velocity-Verlet): the GPU run
    against the oracle's, within the oracle's round-off envelope; n = 20000
    takes the Newton's-third-law force stage."""
    from _gpu_util import dev, state_host, state_tensors
    d = inputs.cloud1024(n=n, seed=9)
    st = inputs.state9(d)
    w = inputs.TWO_PI * 0.2e6
    trap = dict(d["trap"], gamma=0.05 * w * inputs.MASS_40U)
    nsteps = 60 if n <= 1024 else 8
    ref, en_ref, alt, en_alt = _oracle_envelope(oracle, st, d["q"], d["m"], trap, d["dt"], nsteps, every)
    ts = state_tensors(st)
    en = api.md_run(ts, dev(d["q"]), dev(d["m"]), trap, 0.0, d["dt"], nsteps, every=every)
    got = state_host(ts)
    for blk in (slice(0, 3), slice(3, 6), slice(6, 9)):
        D = np.abs(alt[blk] - ref[blk]).max()
        err = np.abs(got[blk] - ref[blk]).max()
        assert err <= 10 * D + 1e-13 * np.abs(ref[blk]).max(), (n, blk, err, D)
    en = en.cpu().numpy()[0]
    assert np.all(np.abs(en - en_ref) <= 10 * np.abs(en_alt - en_ref) + 1e-12 * np.abs(en_ref).max(axis=0))
    # the friction run loses kinetic energy against the friction-free one
    ts0 = state_tensors(st)
    api.md_run(ts0, dev(d["q"]), dev(d["m"]), d["trap"], 0.0, d["dt"], nsteps)
    v_f = np.linalg.norm(got[3:6])
    v_0 = np.linalg.norm(state_host(ts0)[3:6])
    assert v_f < v_0


@pytest.mark.parametrize("n", [1024, 256])
def test_md_run_captured_in_a_hip_graph_replays_bitwise(api, n):
    """The single-run md_run enqueues kernels and device copies only (no
    memset, no host sync), so a caller can capture it in a HIP graph: every
    replay, with eager work in between, equals the eager run bitwise (state
    and energy records).  At 1024 ions the two-launch step, at 256 the
    one-launch step."""
    import torch
    from _gpu_util import dev, state_tensors
    d = inputs.cloud1024(n=n)
    st = inputs.state9(d)
    q, m = dev(d["q"]), dev(d["m"])
    nsteps = 40
    eager = state_tensors(st)
    en_eager = api.md_run(eager, q, m, d["trap"], 0.0, d["dt"], nsteps, every=1).clone()
    ref = torch.stack(eager)
    static = state_tensors(st)
    api.md_run(static, q, m, d["trap"], 0.0, d["dt"], 2, every=1)  # warm-up: workspace, library state
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s0 = torch.stack(state_tensors(st))
    for k in range(9):
        static[k].copy_(s0[k])
    with torch.cuda.graph(g):
        en_static = api.md_run(static, q, m, d["trap"], 0.0, d["dt"], nsteps, every=1)
    for rep in range(3):
        for k in range(9):
            static[k].copy_(s0[k])
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(torch.stack(static), ref), rep
        assert torch.equal(en_static, en_eager), rep
        other = state_tensors(st)  # eager work between replays
        api.md_run(other, q, m, d["trap"], 0.0, d["dt"], 5)
        torch.cuda.synchronize()


@pytest.mark.parametrize("nrun", [1, 3])
def test_energy_records_next_to_the_state_are_not_aliases(api, nrun):
    """Energy records in the same allocation as the state arrays, directly
    before or after them, are accepted and give the results of separate
    buffers (single run and ensemble); records overlapping a state array
    are refused with CB_EINVAL."""
    import torch
    from _gpu_util import dev
    d = inputs.cloud1024(n=900)
    st = inputs.state9(d)
    n = st.shape[1]
    offs = [0, 300, 600, 900] if nrun == 3 else None
    nsteps, every = 6, 2
    nrec = nsteps // every + 1
    q, m = dev(d["q"]), dev(d["m"])
    ref = [dev(st[k]) for k in range(9)]
    en_ref = api.md_run(ref, q, m, d["trap"], 0.0, d["dt"], nsteps, offsets=offs, every=every)
    E = 4 * nrec * nrun
    for where in ("before", "after"):
        buf = torch.zeros(E + 9 * n + E, dtype=torch.float64, device="cuda")
        ts = [buf[E + k * n:E + (k + 1) * n] for k in range(9)]
        for k in range(9):
            ts[k].copy_(dev(st[k]))
        rec = buf[:E] if where == "before" else buf[E + 9 * n:]
        api.md_run(ts, q, m, d["trap"], 0.0, d["dt"], nsteps, offsets=offs, every=every,
                   out=rec.view(nrun, nrec, 4))
        torch.cuda.synchronize()
        assert torch.equal(torch.stack(ts), torch.stack(ref)), where
        assert torch.equal(rec.view(nrun, nrec, 4), en_ref), where
    with pytest.raises(api.CoulombError) as err:
        api.md_run(ts, q, m, d["trap"], 0.0, d["dt"], nsteps, offsets=offs, every=every,
                   out=buf[E + 4 * n - 2:E + 4 * n - 2 + E].view(nrun, nrec, 4))
    assert err.value.status == api.CB_EINVAL


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1000, 4097, 8192])
def test_small_run_path_matches_two_launch_path_and_oracle(api, oracle, n):
    """Runs of at most 8192 ions can take one launch per step (algorithm 3:
    every pair of the run evaluated directly by one wave per 64 ions and
    j-part, then trap, kick and drift; the default up to 384 ions) or the
    two-launch step (algorithm 0).  Both agree to rounding, with and without
    CB_INIT_ACCEL, on an RF trap with friction, energies every other step;
    small runs also against the oracle."""
    import torch
    from _gpu_util import dev, state_host, state_tensors
    g = np.random.Generator(np.random.PCG64(1000 + n))
    trap = dict(inputs.rf_trap(0.0, 0.3, 10e6, 0.2e6), gamma=2e5 * M40)
    sig = inputs.crystal_sigma(max(n, 2), 2 * math.pi * 0.5e6, 2 * math.pi * 0.5e6, trap["wz"])
    st = np.zeros((9, n))
    st[:3] = g.normal(size=(3, n)) * sig[:, None]
    st[3:6] = inputs.maxwell(g, n, 10e-3, M40)
    st[6:9] = g.normal(size=(3, n)) * 1e9  # a_0 used as given without CB_INIT_ACCEL
    q = np.full(n, E)
    q[::5] *= 2.0
    m = np.full(n, M40)
    dt, nsteps, every = 5e-9, 12, 2
    res = {}
    for path in ("small", "two-launch"):
        for init in (True, False):
            if path == "two-launch":
                api.set_config("md_run", n, "fp64", p=1, wg=64, splits=max(1, min(16, n // 64)), algo=0)
            else:
                api.set_config("md_run", n, "fp64", p=1, wg=64, splits=max(1, min(8, n // 32)), algo=3)
            ts = state_tensors(st)
            en = api.md_run(ts, dev(q), dev(m), trap, 0.0, dt, nsteps, every=every, init_accel=init)
            torch.cuda.synchronize()
            api.reset_config("md_run", n, "fp64")
            res[path, init] = (state_host(ts), en.cpu().numpy()[0])
    assert api.poll_flags() == 0
    for init in (True, False):
        a, b = res["small", init], res["two-launch", init]
        for blk in (slice(0, 3), slice(3, 6), slice(6, 9)):
            scale = np.abs(b[0][blk]).max()
            assert np.abs(a[0][blk] - b[0][blk]).max() <= 1e-12 * scale, (n, init, blk)
        assert np.abs(a[1] - b[1]).max() <= 1e-12 * np.abs(b[1]).max(), (n, init)
    if n <= 1000:  # the oracle at full size
        ref, en_ref, _ = oracle.md_run(st, q, m, trap, 0.0, dt, nsteps, every=every)
        got, en = res["small", True]
        for blk in (slice(0, 3), slice(3, 6), slice(6, 9)):
            assert np.abs(got[blk] - ref[blk]).max() <= 1e-11 * np.abs(ref[blk]).max(), (n, blk)
        assert np.abs(en - en_ref).max() <= 1e-11 * np.abs(en_ref).max()


@pytest.mark.parametrize("n,algo", [(300, 3), (300, 0), (1000, 0), (20000, 2)])
def test_rf_drive_with_a_term_and_phase_matches_oracle(api, oracle, n, algo):
    """The explicit RF drive with a DC term and a phase (a != 0, phi != 0) on
    every single-run path: the one-launch step (algorithm 3), the two-launch
    step with the direct kernel (0) and with the Newton's-third-law stage (2),
    against the oracle within its round-off envelope, energies included."""
    from _gpu_util import dev, state_host, state_tensors
    d = inputs.rf32768(n=n, seed=41)
    trap = inputs.rf_trap(0.02, 0.3, 10e6, 0.1e6, phase=0.7)
    st = inputs.state9(d)
    g = np.random.Generator(np.random.PCG64(42))
    st[3:6] = inputs.maxwell(g, n, 10e-3, M40)
    nsteps, every = (24, 4) if n <= 1000 else (6, 3)
    if algo == 3:
        api.set_config("md_run", n, "fp64", p=1, wg=64, splits=4, algo=3)
    elif algo == 0:
        api.set_config("md_run", n, "fp64", p=1, wg=64, splits=max(1, n // 64), algo=0)
    else:
        api.set_config("md_run", n, "fp64", p=4, wg=4, splits=256, algo=2)
    try:
        ref, en_ref, alt, en_alt = _oracle_envelope(oracle, st, d["q"], d["m"], trap, d["dt"], nsteps, every)
        ts = state_tensors(st)
        en = api.md_run(ts, dev(d["q"]), dev(d["m"]), trap, 0.0, d["dt"], nsteps, every=every)
        got = state_host(ts)
    finally:
        api.reset_config("md_run", n, "fp64")
    for blk in (slice(0, 3), slice(3, 6), slice(6, 9)):
        D = np.abs(alt[blk] - ref[blk]).max()
        err = np.abs(got[blk] - ref[blk]).max()
        print(f"[rf a,phi n={n} algo={algo}] block {blk}: err={err:.3e} envelope={D:.3e}", flush=True)
        assert err <= 10 * D + 1e-13 * np.abs(ref[blk]).max(), (blk, err, D)
    en = en.cpu().numpy()[0]
    assert np.all(np.abs(en - en_ref) <= 10 * np.abs(en_alt - en_ref) + 1e-12 * np.abs(en_ref).max(axis=0))
    # the DC term and the phase change the trajectory (the test is not vacuous)
    plain, _, _ = oracle.md_run(st, d["q"], d["m"], inputs.rf_trap(0.0, 0.3, 10e6, 0.1e6), 0.0, d["dt"], nsteps)
    assert np.abs(plain[6:9] - ref[6:9]).max() > 1e3 * np.abs(got[6:9] - ref[6:9]).max()
    assert api.poll_flags() == 0
