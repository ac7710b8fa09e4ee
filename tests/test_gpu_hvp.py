"""GPU Hessian-vector products, autograd double backward, minimiser, Lanczos
normal modes and the checkpointed discrete adjoint, against the oracle, exact
identities and finite differences."""
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


def _cloud(n, seed, charges=(1.0,)):
    g = np.random.Generator(np.random.PCG64(seed))
    pos = g.normal(0.0, 20e-6, size=(3, n))
    return pos, E * g.choice(np.asarray(charges), size=n)


@pytest.mark.parametrize("n,nvec,with_trap", [(1024, 1, False), (1023, 3, True), (777, 8, True), (65, 5, False),
                                              (8192, 2, True), (8192, 8, True), (8192, 4, False), (2, 1, False)])
def test_hvp_matches_oracle(api, oracle, n, nvec, with_trap):
    """Every ion of every vector: the per-ion relative error
    |(Hv)_i - ref_i| / |ref_i| (3-vector norms) against the oracle's exact
    product, like the force parity."""
    from _gpu_util import dev, host
    pos, q = _cloud(n, 40 + n, charges=(1.0, 2.0))
    g = np.random.Generator(np.random.PCG64(n + nvec))
    v = g.normal(size=(nvec, 3, n))
    m = np.full(n, M40)
    trap = inputs.rf_trap(0.02, 0.3, 10e6, 0.1e6, phase=0.4) if with_trap else None
    ref = oracle.hvp(*pos, q, v, m=m if with_trap else None, trap=trap, t=1.3e-8)
    for prec, tol in (("fp64", 1e-12), ("mixed", 1e-8)):
        hv = host(api.coulomb_hvp(dev(pos[0]), dev(pos[1]), dev(pos[2]), dev(q), dev(v),
                                  dev(m) if with_trap else None, trap, 1.3e-8, prec=prec))
        err = np.linalg.norm(hv - ref, axis=1) / np.linalg.norm(ref, axis=1)  # [nvec][n]
        b, i = np.unravel_index(int(np.argmax(err)), err.shape)
        print(f"[hvp n={n} nvec={nvec} {prec}] per-ion max rel {err.max():.3e} (vector {b}, ion {i}), "
              f"rms {np.sqrt(np.mean(err ** 2)):.3e}", flush=True)
        assert err.max() <= tol


HVP_SYM_SHAPES = [(1, 64, 4), (2, 128, 4), (2, 512, 2), (4, 256, 1), (1, 256, 2), (4, 64, 4)]
HVP_SIZES = [2, 65, 129, 130, 257, 1000, 2049, 4097]


@pytest.mark.parametrize("p,jl,nvmax", HVP_SYM_SHAPES)
def test_hvp_symmetric_ragged_sizes(api, oracle, p, jl, nvmax):
    """The Newton's-third-law HVP (each unordered pair once, reactions summed
    over the wave): i-blocks of 64 p, j-segments of jl, at most nvmax vectors
    per pass, ragged blocks and segments, 1, 3, 8 and 7 vectors (passes of
    4, 2 and 1, up to two passes in one launch, with a remainder), mixed
    charges and ions grouped by species, with and without the trap term; every
    ion of every vector against the oracle."""
    from _gpu_util import dev, host
    for k, n in enumerate(HVP_SIZES):
        g = np.random.Generator(np.random.PCG64(700 + n))
        pos = g.normal(0.0, 20e-6, size=(3, n))
        if k % 2:
            q = E * g.choice([1.0, 2.0, -1.0], size=n)
        else:
            q = np.full(n, E)
            q[int(0.6 * n):] = 2.0 * E
        nvec = (1, 3, 8, 7)[k % 4]
        v = g.normal(size=(nvec, 3, n))
        m = np.full(n, M40)
        trap = inputs.rf_trap(0.02, 0.3, 10e6, 0.1e6, phase=0.4) if k % 2 == 0 else None
        eps2 = (1e-7) ** 2 if n % 2 else 0.0
        ref = oracle.hvp(*pos, q, v, m=m if trap else None, trap=trap, t=1.3e-8, eps2=eps2)
        for prec, tol in (("fp64", 1e-12), ("mixed", 1e-8)):
            api.set_config("hvp", n, prec, p=p, wg=nvmax, splits=jl, algo=2)
            try:
                hv = host(api.coulomb_hvp(dev(pos[0]), dev(pos[1]), dev(pos[2]), dev(q), dev(v),
                                          dev(m) if trap else None, trap, 1.3e-8, eps2=eps2, prec=prec))
            finally:
                api.reset_config("hvp", n, prec)
            err = np.linalg.norm(hv - ref, axis=1) / np.linalg.norm(ref, axis=1)
            assert err.max() <= tol, (p, jl, n, nvec, prec, err.max())
    assert api.poll_flags() == 0
    api.clear_workspace_cache()


def test_hvp_default_launch_is_newtons_third_law_at_8192(api):
    for op in ("hvp", "adjoint"):
        cfg = api.get_config(op, 8192, "fp64")
        assert (cfg["algo"], cfg["p"], cfg["wg"], cfg["splits"]) == (2, 2, 4, 128)
        assert api.get_config(op, 4095, "fp64")["algo"] == 0


def test_hvp_exact_identities(api, oracle):
    from _gpu_util import dev, host
    pos, q = _cloud(2000, 5, charges=(1.0, 2.0))
    P = [dev(pos[c]) for c in range(3)]
    F = np.stack([host(t) for t in api.coulomb_forces(*P, dev(q))])
    scale = np.linalg.norm(F, axis=0).max()
    Hr = host(api.coulomb_hvp(*P, dev(q), dev(pos)))
    assert np.abs(Hr - 2.0 * F).max() <= 1e-11 * scale  # degree -1 homogeneity
    for e in np.eye(3):
        Kr = np.cross(e, pos.T).T
        HK = host(api.coulomb_hvp(*P, dev(q), dev(Kr)))
        assert np.abs(HK + np.cross(e, F.T).T).max() <= 1e-11 * scale  # rotation invariance
    g = np.random.Generator(np.random.PCG64(9))
    u, w = g.normal(size=(3, 2000)), g.normal(size=(3, 2000))
    Hu, Hw = host(api.coulomb_hvp(*P, dev(q), dev(u))), host(api.coulomb_hvp(*P, dev(q), dev(w)))
    assert abs(np.sum(u * Hw) - np.sum(w * Hu)) <= 1e-12 * np.abs(u * Hw).sum()


@pytest.mark.parametrize("trap,t", [
    (inputs.rf_trap(0.02, 0.3, 10e6, 0.1e6, phase=0.7), 3.7e-8),
    (inputs.ramp_trap(1.5e6, 0.6e6, 0.15e6, 0.0, 20e-6), 7e-6),
    (inputs.pseudo_trap(1e6, 1e6, 0.2e6), 0.0),
    (None, 0.0),
])
def test_autograd_energy_and_gradient_match_oracle(api, oracle, trap, t):
    """autograd.energy / autograd.gradient (coulomb_trap_grad in the library)
    and the trap constants (cb_trap_k) against the oracle's trap_k, accel,
    coulomb_energy and trap_energy, for an RF drive with a DC term and a
    phase at t != 0, a ramp inside its ramp, a static trap, and no trap."""
    import torch
    from paper_2106_11143_amd import autograd as AG
    from _gpu_util import dev, host
    n = 700
    pos, q = _cloud(n, 6, charges=(1.0, 2.0))
    m = np.full(n, M40)
    mm = dev(m) if trap is not None else None
    if trap is not None:
        k = np.array(AG.trap_k(trap, t))
        kref = oracle.trap_k(trap, t)
        assert np.all(np.abs(k - kref) <= 4 * 2.0 ** -53 * np.abs(kref)), (k, kref)
    r = dev(pos).requires_grad_(True)
    U = AG.energy(r, dev(q), mm, trap, t)
    (G,) = torch.autograd.grad(U, r, create_graph=True)
    G2 = AG.gradient(dev(pos), dev(q), mm, trap, t)
    assert torch.equal(G.detach(), G2)
    if trap is not None:
        Gref = -m[None, :] * oracle.accel(*pos, q, m, trap, t)
        Uref = oracle.coulomb_energy(*pos, q)[0] + oracle.trap_energy(*pos, m, trap, t)
    else:
        Gref = -np.stack(oracle.forces(*pos, q))
        Uref = oracle.coulomb_energy(*pos, q)[0]
    err = np.linalg.norm(host(G.detach()) - Gref, axis=0) / np.linalg.norm(Gref, axis=0)
    print(f"[autograd trap={None if trap is None else trap['kind']}] gradient max rel {err.max():.3e}, "
          f"energy rel {abs(float(U.detach()) - Uref) / abs(Uref):.3e}", flush=True)
    assert err.max() <= 1e-12
    assert abs(float(U.detach()) - Uref) <= 1e-12 * abs(Uref)
    # double backward is the HVP kernel
    w = dev(np.random.Generator(np.random.PCG64(2)).normal(size=(3, n)))
    (Hw,) = torch.autograd.grad(G, r, grad_outputs=w)
    direct = api.coulomb_hvp(*[dev(pos[c]) for c in range(3)], dev(q), w, mm, trap, t)
    assert torch.equal(Hw, direct)


def _crystal(n, fr, fz, seed=1):
    import torch
    from paper_2106_11143_amd import drivers
    from _gpu_util import dev
    trap = inputs.pseudo_trap(fr, fr, fz)
    sig = inputs.crystal_sigma(n, trap["wx"], trap["wy"], trap["wz"])
    g = np.random.Generator(np.random.PCG64(seed))
    r0 = dev(g.normal(size=(3, n)) * sig[:, None])
    q, m = dev(np.full(n, E)), dev(np.full(n, M40))
    r, info = drivers.minimise(r0, q, m, trap, ftol_rel=1e-12)
    return r, q, m, trap, info


def test_minimiser_and_lanczos_normal_modes(api):
    import torch
    from paper_2106_11143_amd import drivers
    n = 300
    r, q, m, trap, info = _crystal(n, 1.0e6, 0.05e6)
    print(f"[minimise n={n}] {info}", flush=True)
    assert info["fmax_rel"] <= 1e-12
    lam, vecs, res, info = drivers.lanczos_lowest(r, q, m, trap, k=32, block=8, maxdim=1200)
    wz2 = trap["wz"] ** 2
    lam = lam.cpu().numpy()
    print(f"[lanczos] lowest/wz^2: {np.round(lam[:8] / wz2, 6)} max res {float(res.max()):.2e}", flush=True)
    # the rotation about z (wx = wy) is a zero mode and the axial centre-of-mass
    # mode has exactly wz^2 (Kohn), for any crystal
    assert abs(lam[0]) <= 1e-8 * wz2
    assert np.min(np.abs(lam - wz2)) <= 1e-8 * wz2
    assert np.all(np.diff(lam) >= -1e-9 * wz2)


def test_trajectory_gradient_matches_oracle_and_fd(api, oracle):
    import torch
    from paper_2106_11143_amd import drivers
    from _gpu_util import dev
    d = inputs.crystal8192(n=96, seed=21)
    trap = d["trap"]
    st = inputs.state9(d)
    q, m = dev(d["q"]), dev(d["m"])
    dt, nsteps = 1e-9, 120
    L, g, info = drivers.traj_grad(dev(st), q, m, trap, dt, nsteps, checkpoint_every=50)
    Lr, gr = oracle.msd_grad(st[:6], d["q"], d["m"], trap, dt, nsteps)
    g = g.cpu().numpy()
    print(f"[traj_grad] L {L:.6e} vs {Lr:.6e}; grad {g} vs {gr}", flush=True)
    assert L == pytest.approx(Lr, rel=1e-10)
    assert np.allclose(g, gr, rtol=1e-8, atol=1e-12 * np.abs(gr).max())

    def loss(tr):
        s = [dev(st[k]) for k in range(9)]
        api.md_run(s, q, m, tr, 0.0, dt, nsteps)
        return float(sum(((s[c] - dev(st[c])) ** 2).sum() for c in range(3))) / 96

    for c, key in enumerate(("wx", "wz")):
        h = 1e-6 * trap[key]
        tp, tm = dict(trap), dict(trap)
        tp[key] += h
        tm[key] -= h
        fd = (loss(tp) - loss(tm)) / (2 * h)
        gc = g[0] if key == "wx" else g[2]
        assert gc == pytest.approx(fd, rel=1e-5)


def test_damped_md_minimiser_reaches_the_lbfgs_chain(api):
    """Damped molecular dynamics (md_run with the friction term) and L-BFGS
    relax the same start to the same linear chain (a unique minimum)."""
    from paper_2106_11143_amd import drivers
    from _gpu_util import dev
    n = 10
    trap = inputs.pseudo_trap(5.0e6, 5.0e6, 0.2e6)
    g = np.random.Generator(np.random.PCG64(4))
    r0 = dev(g.normal(size=(3, n)) * np.array([1e-7, 1e-7, 20e-6])[:, None])
    q, m = dev(np.full(n, E)), dev(np.full(n, M40))
    ra, ia = drivers.minimise(r0, q, m, trap, ftol_rel=1e-10)
    rb, ib = drivers.minimise(r0, q, m, trap, ftol_rel=1e-9, method="damped", max_iter=400000)
    print(f"[minimise lbfgs] {ia}\n[minimise damped] {ib}", flush=True)
    assert ib["fmax_rel"] <= 1e-9
    za = np.sort(ra[2].cpu().numpy())
    zb = np.sort(rb[2].cpu().numpy())
    assert np.max(np.abs(za - zb)) <= 1e-7 * np.max(np.abs(za))
    assert np.max(np.abs(rb[:2].cpu().numpy())) <= 1e-9 * np.max(np.abs(za))


@pytest.mark.parametrize("p,jl", [(1, 64), (2, 128)])
def test_trajectory_gradient_on_the_symmetric_hvp(api, oracle, p, jl):
    """md_adjoint_step with its Coulomb product on the Newton's-third-law
    tiles (the default from 4096 ions, forced here at 300): the checkpointed
    adjoint gradient against the oracle's discrete adjoint."""
    from paper_2106_11143_amd import drivers
    from _gpu_util import dev
    n = 300
    d = inputs.crystal8192(n=n, seed=22)
    trap = d["trap"]
    st = inputs.state9(d)
    dt, nsteps = 1e-9, 80
    api.set_config("adjoint", n, "fp64", p=p, wg=1, splits=jl, algo=2)
    try:
        L, g, _ = drivers.traj_grad(dev(st), dev(d["q"]), dev(d["m"]), trap, dt, nsteps, checkpoint_every=25)
    finally:
        api.reset_config("adjoint", n, "fp64")
    Lr, gr = oracle.msd_grad(st[:6], d["q"], d["m"], trap, dt, nsteps)
    g = g.cpu().numpy()
    print(f"[traj_grad sym p={p} jl={jl}] L {L:.6e} vs {Lr:.6e}; grad {g} vs {gr}", flush=True)
    assert L == pytest.approx(Lr, rel=1e-10)
    assert np.allclose(g, gr, rtol=1e-8, atol=1e-12 * np.abs(gr).max())
