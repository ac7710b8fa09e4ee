"""Host-side driver logic that needs no GPU."""
import numpy as np

from paper_2106_11143_amd.drivers import count_defects


def _zigzag(n, kinks_at=(), amp=1e-6, spacing=5e-6, seed=0):
    z = np.arange(n) * spacing
    s = np.array([(-1) ** k for k in range(n)], dtype=float)
    for k in kinks_at:  # flip the pattern after position k: one domain wall
        s[k + 1:] *= -1
    g = np.random.Generator(np.random.PCG64(seed))
    theta = 0.7
    x = amp * s * np.cos(theta) + 1e-9 * g.normal(size=n)
    y = amp * s * np.sin(theta) + 1e-9 * g.normal(size=n)
    perm = g.permutation(n)  # input order must not matter
    return x[perm], y[perm], z[perm]


def test_perfect_zigzag_has_no_defect():
    assert count_defects(*_zigzag(40)) == 0


def test_domain_walls_are_counted():
    assert count_defects(*_zigzag(40, kinks_at=(10,))) == 1
    assert count_defects(*_zigzag(60, kinks_at=(10, 30, 31))) == 3


def test_tiny_chains():
    assert count_defects([0.0, 1.0], [0.0, 0.0], [0.0, 1.0]) == 0


def test_block_lanczos_against_dense_eigensolver(oracle):
    """The Lanczos driver's algorithm, with the oracle's HVP as the operator,
    reproduces the lowest eigenvalues of the dense mass-weighted Hessian."""
    import torch
    from paper_2106_11143_amd import drivers, inputs

    n = 60
    g = np.random.Generator(np.random.PCG64(4))
    trap = inputs.pseudo_trap(1e6, 1e6, 0.3e6)
    pos = g.normal(size=(3, n)) * inputs.crystal_sigma(n, trap["wx"], trap["wy"], trap["wz"])[:, None]
    q = np.full(n, inputs.E_CHARGE)
    m = np.full(n, inputs.MASS_40U) * (1.0 + 0.1 * g.random(n))

    def hvp(V):
        return torch.as_tensor(oracle.hvp(*pos, q, V.numpy(), m=m, trap=trap))

    cols = [oracle.hvp(*pos, q, e.reshape(3, n), m=m, trap=trap).reshape(-1) for e in np.eye(3 * n)]
    H = np.array(cols).T
    sm = np.sqrt(np.tile(m, 3))
    ref = np.linalg.eigvalsh((H / sm[:, None]) / sm[None, :])
    r = torch.as_tensor(pos)
    lam, vecs, res, info = drivers.lanczos_lowest(r, torch.as_tensor(q), torch.as_tensor(m), trap, k=6, block=4,
                                                  maxdim=3 * n, hvp=hvp, check_every=5)
    scale = np.abs(ref).max()
    assert np.abs(lam.numpy() - ref[:6]).max() <= 1e-10 * scale
    # Ritz vectors are eigenvectors of the mass-weighted operator
    V = vecs.numpy().reshape(6, -1)
    Av = np.stack([((H @ (v / sm)) / sm) for v in V])
    assert np.abs(Av - lam.numpy()[:, None] * V).max() <= 1e-8 * scale


def test_block_lanczos_resolves_exactly_degenerate_modes():
    """An operator whose every eigenvalue is doubly degenerate (two identical
    decoupled copies, as the x/y modes of a cylindrically symmetric trap):
    the Ritz values come in equal pairs and the Ritz vectors stay orthonormal
    eigenvectors."""
    import torch
    from paper_2106_11143_amd import drivers

    n = 20  # 3n = 60 = two copies of a 30-dimensional operator
    g = np.random.Generator(np.random.PCG64(8))
    lam0 = np.sort(g.uniform(1.0, 50.0, 30))
    Q0 = np.linalg.qr(g.normal(size=(30, 30)))[0]
    D = (Q0 * lam0) @ Q0.T
    H = np.zeros((60, 60))
    H[:30, :30] = D
    H[30:, 30:] = D
    P = np.linalg.qr(g.normal(size=(60, 60)))[0]  # hide the block structure
    H = P @ H @ P.T

    def hvp(V):
        B = V.shape[0]
        return torch.as_tensor((V.numpy().reshape(B, 60) @ H).reshape(B, 3, n))

    r = torch.zeros(3, n, dtype=torch.float64)
    ones = torch.ones(n, dtype=torch.float64)
    lam, vecs, res, info = drivers.lanczos_lowest(r, ones, ones, {"kind": 0}, k=6, block=4, maxdim=60, hvp=hvp,
                                                  check_every=3)
    lam = lam.numpy()
    ref = np.repeat(lam0[:3], 2)
    assert np.abs(lam - ref).max() <= 1e-10 * lam0.max()
    V = vecs.numpy().reshape(6, -1)
    assert np.abs(V @ V.T - np.eye(6)).max() <= 1e-9
    assert np.abs(V @ H - lam[:, None] * V).max() <= 1e-8 * lam0.max()


def test_lbfgs_direction_matches_the_two_loop_recursion():
    """The L-BFGS inverse-Hessian product (two-loop recursion over stored
    inner products) against the two-loop recursion written out on vectors, on curvature pairs of a random
    symmetric positive definite quadratic; with one pair and H itself
    quadratic, H s = y is reproduced (the secant condition)."""
    import torch
    from paper_2106_11143_amd import drivers
    g_ = np.random.default_rng(5)
    n, k = 40, 7
    B = g_.standard_normal((3 * n, 3 * n))
    H = B @ B.T + 3 * n * np.eye(3 * n)
    S = [torch.as_tensor(g_.standard_normal((3, n))) for _ in range(k)]
    Y = [torch.as_tensor((H @ s.numpy().reshape(-1)).reshape(3, n)) for s in S]
    g = torch.as_tensor(g_.standard_normal((3, n)))
    got = drivers.lbfgs_direction(g, S, Y, 0.1)
    z, al = g.clone(), []
    for s, y in reversed(list(zip(S, Y))):
        a = float((s * z).sum()) / float((y * s).sum())
        al.append(a)
        z = z - a * y
    z = z * float((S[-1] * Y[-1]).sum()) / float((Y[-1] * Y[-1]).sum())
    for (s, y), a in zip(zip(S, Y), reversed(al)):
        z = z + (a - float((y * z).sum()) / float((y * s).sum())) * s
    assert torch.allclose(got, -z, rtol=1e-10, atol=1e-12 * float(z.abs().max()))
    assert torch.equal(drivers.lbfgs_direction(g, [], [], 0.1), -0.1 * g)
    # secant condition of the newest pair: H y_last = s_last
    hy = -drivers.lbfgs_direction(Y[-1], S, Y, 0.1)
    assert torch.allclose(hy, S[-1], rtol=1e-9, atol=1e-12 * float(S[-1].abs().max()))


def _two_loop(g, S, Y):
    z, al = g.clone(), []
    for s, y in reversed(list(zip(S, Y))):
        a = float((s * z).sum()) / float((y * s).sum())
        al.append(a)
        z = z - a * y
    z = z * float((S[-1] * Y[-1]).sum()) / float((Y[-1] * Y[-1]).sum())
    for (s, y), a in zip(zip(S, Y), reversed(al)):
        z = z + (a - float((y * z).sum()) / float((y * s).sum())) * s
    return -z


def test_lbfgs_memory_keeps_the_newest_pairs_with_positive_curvature():
    """A memory of 3 fed 6 candidate pairs, one with s . y < 0, along with a
    changing gradient: it keeps the 3 newest accepted pairs (slots reused
    oldest first) and gives the two-loop recursion's direction for them and
    the last gradient; after clear() it gives -h0 g."""
    import torch
    from paper_2106_11143_amd import drivers
    g_ = np.random.default_rng(9)
    n = 30
    B = g_.standard_normal((3 * n, 3 * n))
    H = B @ B.T + 3 * n * np.eye(3 * n)
    mem = drivers.LbfgsMemory((3, n), 3, "cpu", torch.float64)
    g = torch.as_tensor(g_.standard_normal((3, n)))
    mem.set_gradient(g)
    kept_s, kept_y = [], []
    for k in range(6):
        s = torch.as_tensor(g_.standard_normal((3, n)))
        y = torch.as_tensor((H @ s.numpy().reshape(-1)).reshape(3, n))
        if k == 3:
            y = -y  # negative curvature: rejected
        else:
            kept_s.append(s)
            kept_y.append(y)
        g = torch.as_tensor(g_.standard_normal((3, n)))
        mem.absorb(mem.load(g, s, y).numpy())
    assert len(mem.order) == 3
    got = mem.direction(0.1)
    ref = _two_loop(g, kept_s[-3:], kept_y[-3:])
    assert torch.allclose(got, ref, rtol=1e-10, atol=1e-12 * float(ref.abs().max()))
    mem.clear()
    assert torch.equal(mem.direction(0.1), -0.1 * g)


def test_split_k_product_equals_plain_product():
    """A^T W by blocks of K summed (Lanczos reorthogonalisation) against the
    plain product: K a multiple of the block count and not, a column slice of
    a wider matrix, and K below one block."""
    import torch
    from paper_2106_11143_amd import drivers
    g_ = torch.Generator().manual_seed(3)
    for K in (24576, 900, 40):
        Q = torch.randn(K, 130, dtype=torch.float64, generator=g_)
        W = torch.randn(K, 8, dtype=torch.float64, generator=g_)
        for c in (8, 57, 130):
            ref = Q[:, :c].T @ W
            got = drivers._tsmm(Q[:, :c], W)
            assert got.shape == ref.shape
            assert torch.allclose(got, ref, rtol=0, atol=1e-13 * float(ref.abs().max()) * (K ** 0.5))


def test_band_ritz_shift_invert_matches_dense_eigensolver():
    """The banded Ritz solve of Lanczos above the dense size limit (shift and
    invert below a certified shift) against the dense eigensolver, on a band
    of width 8 whose spectrum has exactly degenerate pairs (two decoupled
    copies) and negative eigenvalues below a zero mode."""
    from paper_2106_11143_amd import drivers
    g = np.random.Generator(np.random.PCG64(12))
    b, n0 = 8, 450
    band = g.normal(size=(b + 1, n0))
    band[0] += np.linspace(-3.0, 40.0, n0)  # a few negative eigenvalues at the bottom
    two = np.concatenate([band, band], axis=1)
    for d in range(1, b + 1):
        two[d, n0 - d:n0] = 0.0  # no coupling between the copies
    n = 2 * n0
    T = np.zeros((n, n))
    for d in range(b + 1):
        idx = np.arange(n - d)
        T[idx + d, idx] = two[d, :n - d]
        T[idx, idx + d] = two[d, :n - d]
    ref = np.linalg.eigvalsh(T)[:32]
    assert ref[0] < 0.0 and np.abs(ref[0::2] - ref[1::2]).max() <= 1e-10 * np.abs(ref).max()
    w, V = drivers._band_ritz(two, 32, dense_max=64)
    scale = np.abs(T).sum(axis=0).max()
    assert np.abs(w - ref).max() <= 1e-12 * scale
    assert np.abs(V.T @ V - np.eye(32)).max() <= 1e-10
    assert np.abs(T @ V - V * w).max() <= 1e-10 * scale
    w2, _ = drivers._band_ritz(two, 32)  # dense path
    assert np.abs(w2 - ref).max() <= 1e-12 * scale
