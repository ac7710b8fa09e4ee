"""Drivers built on the library's entry points (support code around the hot
path; every force, energy, Hessian product and integration step runs in the
HIP kernels, torch only supplies element-wise glue and the small dense
algebra of Lanczos).

- minimise: L-BFGS with Hessian-vector Newton step lengths (default), FIRE
  (Bitzek et al., PRL 97, 170201 (2006)) or damped molecular dynamics (the
  friction term), to the Coulomb crystal of a trap.
- lanczos_lowest: block Lanczos with full reorthogonalisation on the
  mass-weighted Hessian M^-1/2 H M^-1/2 (eigenvalues = squared normal-mode
  angular frequencies), several vectors per HVP kernel pass.
- traj_grad: d(mean-square displacement after T steps)/d(wx, wy, wz) by the
  discrete adjoint of velocity-Verlet with checkpointed recomputation.
- count_defects: kink count of a quasi-one-dimensional zigzag chain.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import api


def _rows(r):
    return r[0].contiguous(), r[1].contiguous(), r[2].contiguous()


def total_force(r, q, m, trap, t=0.0, eps2=0.0, prec="fp64"):
    """Coulomb + trap force (3, n): minus the gradient the library computes."""
    g, _ = api.coulomb_trap_grad(*_rows(r), q, m, trap, t, eps2, prec)
    return g.neg_()


def _force_scale(m, trap):
    k = api.trap_k(trap, 0.0)
    wmax = math.sqrt(max(k))
    e2kc = 2.307077552e-28  # k_C e^2 (J m), only for the stopping scale
    a = (3.0 * e2kc / (float(m.mean()) * wmax * wmax)) ** (1.0 / 3.0)
    return e2kc / (a * a), a, wmax


def minimise(r, q, m, trap, eps2=0.0, ftol_rel=1e-10, max_iter=100000, method="lbfgs", memory=20):
    """Relaxes positions r (3, n) (copied) to a minimum of U_C + U_trap.

    method "lbfgs": limited-memory BFGS (two-loop recursion, `memory` pairs)
    whose step length along each direction p is the Newton step
    -(g.p)/(p.H p), with H p from the HVP kernel, capped at 0.2 ion spacings
    per ion.  method "fire": FIRE.  method "damped": damped molecular
    dynamics, i.e. md_run with eq. (1)'s friction term, Gamma = 2 m w_min
    (critical damping of the slowest trap axis), in chunks of steps (max_iter
    counts steps).  Stops when max_i |F_i| <= ftol_rel * k_C e^2 / a^2,
    a = (3 k_C e^2 / (m w_max^2))^(1/3).  Returns (r_min, info)."""
    r = r.clone()
    fscale, a, wmax = _force_scale(m, trap)
    minv = 1.0 / m.reshape(1, -1)
    tol = ftol_rel * fscale
    g = -total_force(r, q, m, trap, 0.0, eps2)
    it = 0
    if method == "damped":
        k = api.trap_k(trap, 0.0)
        wmin = math.sqrt(min(k))
        damped = dict(trap, gamma=2.0 * wmin * float(m.mean()))
        dt = 0.05 / wmax
        chunk = max(20, int(0.5 / (wmin * dt)))
        st = [r[c].contiguous() for c in range(3)] + [torch.zeros_like(r[0]) for _ in range(6)]
        first = True
        while it < max_iter:
            if float(g.norm(dim=0).max()) <= tol:
                break
            api.md_run(st, q, m, damped, 0.0, dt, chunk, eps2=eps2, init_accel=first)
            first = False
            it += chunk
            r = torch.stack(st[:3])
            g = -total_force(r, q, m, trap, 0.0, eps2)
    elif method == "fire":
        v = torch.zeros_like(r)
        dt_max, dt = 0.2 / wmax, 0.05 / wmax
        alpha, n_pos = 0.1, 0
        for it in range(max_iter):
            if float(g.norm(dim=0).max()) <= tol:
                break
            v = v - dt * g * minv
            P = -float((g * v).sum())
            if P > 0:
                v = (1 - alpha) * v - alpha * (v.norm() / g.norm()) * g
                n_pos += 1
                if n_pos > 5:
                    dt = min(dt * 1.1, dt_max)
                    alpha *= 0.99
            else:
                v.zero_()
                dt *= 0.5
                alpha, n_pos = 0.1, 0
            r = r + dt * v
            g = -total_force(r, q, m, trap, 0.0, eps2)
    else:
        grad = lambda r: api.coulomb_trap_grad(*_rows(r), q, m, trap, 0.0, eps2, "fp64")[0]
        mem = LbfgsMemory(g.shape, memory, g.device, g.dtype)
        mem.set_gradient(g)
        h0 = 1.0 / (float(m.mean()) * wmax * wmax)
        cap = 0.2 * a
        fmax = float(g.norm(dim=0).max())
        hvp = lambda v: api.coulomb_hvp(*_rows(r), q, v, m, trap, 0.0, eps2)
        for it in range(max_iter):
            if fmax <= tol:
                break
            p = mem.direction(h0)
            Hp = hvp(p)
            gp, pHp = torch.stack([(g * p).sum(), (p * Hp).sum()]).tolist()
            if gp >= 0:  # not a descent direction: restart from steepest descent
                mem.clear()
                p = -h0 * g
                Hp = hvp(p)
                gp, pHp = torch.stack([(g * p).sum(), (p * Hp).sum()]).tolist()
            step = (-gp / pHp if pHp > 0 else 1.0) * p
            step = step * torch.clamp(cap / step.norm(dim=0).max(), max=1.0)  # at most `cap` per ion
            r = r + step
            gn = grad(r)
            D = mem.load(gn, step, gn - g)
            host = torch.cat([D.reshape(-1), gn.norm(dim=0).max().reshape(1)]).cpu().numpy()
            fmax = float(host[-1])
            mem.absorb(host[:-1].reshape(D.shape))  # keeps the pair if s . y > 0
            g = gn
    info = {"method": method, "iters": it, "fmax_rel": float(g.norm(dim=0).max()) / fscale, "force_scale": fscale}
    return r, info


class LbfgsMemory:
    """The newest (at most m) curvature pairs (s_i, y_i), s_i . y_i > 0, of
    L-BFGS as columns of one device matrix W (3n, 2m + 3): s in slots
    [0, m), y in [m, 2m), then the current gradient g and the newest
    candidate pair.  Their inner products (s_i . y_k, y_i . y_k, s_i . g,
    y_i . g) are kept on the host and refreshed by one split-K product
    W^T [g s y] per iteration, so that the two-loop recursion (Nocedal and
    Wright, Algorithm 7.4) runs on host scalars and -H g is one
    matrix-vector product with W.  The recursion is unchanged; each of its
    dot products is expanded over the stored pairs' inner products."""

    def __init__(self, shape, m, device, dtype):
        self.shape, self.m = tuple(shape), m
        self.W = torch.zeros(math.prod(self.shape), 2 * m + 3, dtype=dtype, device=device)
        self.order = []  # slots in use, oldest first
        self.SY = np.zeros((m, m))  # SY[i, k] = s_i . y_k
        self.YY = np.zeros((m, m))  # YY[i, k] = y_i . y_k
        self.Sg = np.zeros(m)
        self.Yg = np.zeros(m)
        pin = self.W.is_cuda
        self.c = torch.zeros(2 * m + 3, dtype=dtype, pin_memory=pin)  # coefficients, host side
        self.c_np = self.c.numpy()

    def clear(self):
        self.order = []

    def set_gradient(self, g):
        """Stores g without products (enough while no pair is held)."""
        self.W[:, 2 * self.m] = g.reshape(-1)
        self.order = []

    def load(self, g, s, y):
        """Stores the gradient g and the candidate pair (s, y); returns the
        device products W^T [g s y], (2m + 3, 3), for absorb()."""
        m, W = self.m, self.W
        W[:, 2 * m] = g.reshape(-1)
        W[:, 2 * m + 1] = s.reshape(-1)
        W[:, 2 * m + 2] = y.reshape(-1)
        return _tsmm(W, W[:, 2 * m:])

    def absorb(self, D):
        """Takes the products of load() (host array): refreshes s_i . g and
        y_i . g, and keeps the candidate pair if s . y > 0 (the oldest pair
        makes room when m are held)."""
        m = self.m
        for i in self.order:
            self.Sg[i], self.Yg[i] = D[i, 0], D[m + i, 0]
        if not D[2 * m + 1, 2] > 0:
            return
        if len(self.order) == m:
            slot = self.order.pop(0)
        else:
            slot = min(set(range(m)) - set(self.order))
        self.W[:, slot] = self.W[:, 2 * m + 1]
        self.W[:, m + slot] = self.W[:, 2 * m + 2]
        for i in self.order:
            self.SY[i, slot] = D[i, 2]  # s_i . y
            self.SY[slot, i] = D[m + i, 1]  # s . y_i
            self.YY[i, slot] = self.YY[slot, i] = D[m + i, 2]
        self.SY[slot, slot], self.YY[slot, slot] = D[2 * m + 1, 2], D[2 * m + 2, 2]
        self.Sg[slot], self.Yg[slot] = D[2 * m + 1, 0], D[2 * m + 2, 0]
        self.order.append(slot)

    def direction(self, h0):
        """-H g, with H_0 = gamma I, gamma = s.y / y.y of the newest pair (h0
        without pairs)."""
        m, W = self.m, self.W
        if not self.order:
            return (-h0 * W[:, 2 * m]).reshape(self.shape)
        o = np.asarray(self.order)
        k = len(o)
        SY, YY = self.SY[np.ix_(o, o)], self.YY[np.ix_(o, o)]
        rho = 1.0 / np.diag(SY)
        # first loop, newest first: alpha_t = rho_t s_t . (g - sum_{u>t} alpha_u y_u)
        al = np.zeros(k)
        for t in range(k - 1, -1, -1):
            al[t] = rho[t] * (self.Sg[o[t]] - SY[t, t + 1:] @ al[t + 1:])
        gam = SY[-1, -1] / YY[-1, -1]
        # z = gam (g - sum_u alpha_u y_u); second loop, oldest first:
        # beta_t = rho_t y_t . z, then z += (alpha_t - beta_t) s_t
        yq = self.Yg[o] - YY @ al
        be = np.zeros(k)
        for t in range(k):
            be[t] = rho[t] * (gam * yq[t] + (al[:t] - be[:t]) @ SY[:t, t])
        # the pinned buffer is rewritten only after the previous copy was
        # awaited (every iteration reads products back in between)
        c = self.c_np
        c[:] = 0.0
        c[2 * m] = gam
        c[o] = al - be
        c[m + o] = -gam * al
        return -(W @ self.c.to(W.device, non_blocking=True)).reshape(self.shape)


def lbfgs_direction(g, S, Y, h0):
    """-H g for the L-BFGS inverse-Hessian approximation H built from the
    curvature pairs (s_i, y_i), oldest first (s_i . y_i > 0), with H_0 =
    gamma I, gamma = s.y / y.y of the newest pair (h0 without pairs); the
    two-loop recursion of LbfgsMemory."""
    mem = LbfgsMemory(g.shape, max(1, len(S)), g.device, g.dtype)
    mem.set_gradient(g)
    for s, y in zip(S, Y):
        mem.absorb(mem.load(g, s, y).cpu().numpy())
    return mem.direction(h0)


def _band_ritz(band, k, dense_max=512):
    """Lowest k eigenpairs of the symmetric banded matrix T given in lower
    form, band[d, c] = T[c + d, c].  Up to dense_max rows: the dense
    symmetric eigensolver.  Beyond: shift-and-invert Lanczos (ARPACK, through
    scipy's eigsh) around a shift sigma certified below the spectrum by a
    banded Cholesky factorisation of T - sigma I, so that the k eigenvalues
    of (T - sigma I)^-1 of largest magnitude belong to the k lowest of T.
    Each solve costs O(n b) after one sparse LU, where reducing the band to
    tridiagonal form (the banded eigenvalue solver) costs O(n^2 b)."""
    from scipy.linalg import LinAlgError, cholesky_banded
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla

    b, n = band.shape[0] - 1, band.shape[1]
    T = sp.diags([band[d, :n - d] for d in range(b + 1)], list(range(0, -b - 1, -1)), shape=(n, n))
    T = (T + sp.tril(T, -1).T).tocsc()
    if n <= max(dense_max, 3 * k):
        w, V = np.linalg.eigh(T.toarray())
        return w[:k], V[:, :k]
    scale = float(np.abs(band).sum(axis=0).max())  # bound on |T| (Gershgorin)
    sigma = -1e-9 * scale
    for _ in range(12):  # reaches -1e2 scale, below every eigenvalue
        shifted = band.copy()
        shifted[0] -= sigma
        try:
            cholesky_banded(shifted, lower=True)
            break
        except LinAlgError:
            sigma *= 10.0
    v0 = np.random.default_rng(0).standard_normal(n)
    w, V = sla.eigsh(T, k=k, sigma=sigma, which="LM", v0=v0, tol=0)
    o = np.argsort(w)
    return w[o], V[:, o]


def _tsmm(A, W, P=64):
    """A^T W for a tall A (K, c) -- also a column slice of a wider matrix --
    and W (K, b).  K is cut into P blocks whose products run as one batched
    GEMM and are then summed: a single GEMM with K ~ 1e4 and a small output
    runs on one workgroup's worth of the chip and takes milliseconds (2.6 ms
    for 8 x 8 at K = 24576 on MI355X, 0.03 ms this way)."""
    K = A.shape[0]
    K0 = K // P * P
    if K0 == 0:
        return A.T @ W
    out = torch.bmm(W[:K0].reshape(P, K0 // P, W.shape[1]).transpose(1, 2).contiguous(),
                    A[:K0].reshape(P, K0 // P, A.shape[1])).sum(0).T
    if K0 < K:
        out = out + A[K0:].T @ W[K0:]
    return out


def _chol_qr2(W, G):
    """W = Q R for a tall W (K, b) with Gram matrix G = W^T W (host): two
    rounds of Cholesky QR (R_1 = chol(G), W R_1^-1, and again on the result),
    which give Q orthonormal to rounding while cond(W) stays below about
    1e7.  A Gram matrix that is not safely positive definite (a nearly
    rank-deficient block) goes to Householder QR instead.  Returns (Q on W's
    device, R on the host)."""
    def chol(G):
        L = np.linalg.cholesky(0.5 * (G + G.T))  # raises if not positive definite
        d = np.abs(np.diag(L))
        if d.min() <= 1e-7 * d.max():
            raise np.linalg.LinAlgError("ill-conditioned block")
        return L.T

    try:
        R1 = chol(G)
        Q1 = W @ torch.as_tensor(np.linalg.inv(R1), dtype=W.dtype, device=W.device)
        R2 = chol(_tsmm(Q1, Q1).cpu().numpy())
        return Q1 @ torch.as_tensor(np.linalg.inv(R2), dtype=W.dtype, device=W.device), R2 @ R1
    except np.linalg.LinAlgError:
        Qh, Rh = torch.linalg.qr(W)
        return Qh, Rh.cpu().numpy()


def lanczos_lowest(r, q, m, trap, k=32, block=8, maxdim=12000, eps2=0.0, seed=0, tol=1e-8, check_every=20,
                   hvp=None):
    """Lowest k eigenpairs of the mass-weighted Hessian M^-1/2 H M^-1/2 of
    U_C + U_trap at r (eigenvalues = squared mode angular frequencies).

    Block Lanczos (`block` vectors per HVP kernel pass) with full
    reorthogonalisation against a preallocated basis.  The projected matrix
    is block tridiagonal, i.e. banded with bandwidth `block`, so its lowest
    Ritz pairs come from banded solves (_band_ritz).  Stops when every
    wanted Ritz residual |A u - theta u| is below tol * theta_k, or when the
    basis reaches maxdim.  `hvp(V)` may replace the kernel call
    (V: (B, 3, n) -> H V).  Returns (eigenvalues (k,), vectors (k, 3, n) in
    mass-weighted coordinates, residual norms (k,), info)."""

    n = r.shape[1]
    N3 = 3 * n
    dev, dt = r.device, r.dtype
    sm = torch.sqrt(m).reshape(1, -1)
    if hvp is None:
        hvp = lambda vv: api.coulomb_hvp(*_rows(r), q, vv.contiguous(), m, trap, 0.0, eps2)

    def A(V):  # (N3, B) -> (N3, B)
        B = V.shape[1]
        return (hvp((V.T.reshape(B, 3, n) / sm).contiguous()) / sm).reshape(B, N3).T

    maxdim = max(block, min(maxdim, N3) // block * block)
    nblk = maxdim // block
    Q = torch.empty(N3, maxdim + block, dtype=dt, device=dev)
    g = torch.Generator(device="cpu").manual_seed(seed)
    Q[:, :block] = torch.linalg.qr(torch.randn(N3, block, generator=g, dtype=dt))[0].to(dev)
    band = np.zeros((block + 1, maxdim))  # band[d, c] = T[c + d, c]
    Bprev = None
    theta = S = res = None
    used = 0
    next_check = check_every
    for j in range(nblk):
        c0, c1 = j * block, (j + 1) * block
        Qj = Q[:, c0:c1]
        W = A(Qj)
        if Bprev is not None:
            W = W - Q[:, c0 - block:c0] @ Bprev.T
        Aj = _tsmm(Qj, W)
        Aj = 0.5 * (Aj + Aj.T)
        W = W - Qj @ Aj
        # full reorthogonalisation against the basis; a second pass only where
        # the first removed more than half of a column's squared norm
        # (Daniel, Gragg, Kaufman and Stewart's criterion)
        n0 = (W * W).sum(0)
        W = W - Q[:, :c1] @ _tsmm(Q[:, :c1], W)
        host = torch.cat([Aj.reshape(-1), n0, _tsmm(W, W).reshape(-1)]).cpu().numpy()
        Ah = host[:block * block].reshape(block, block)
        n0h = host[block * block:block * block + block]
        G = host[block * block + block:].reshape(block, block)
        if np.any(np.diag(G) < 0.5 * n0h):
            W = W - Q[:, :c1] @ _tsmm(Q[:, :c1], W)
            G = _tsmm(W, W).cpu().numpy()
        Qn, Bh = _chol_qr2(W, G)
        Q[:, c1:c1 + block] = Qn
        Bj = torch.as_tensor(Bh, dtype=dt, device=dev)
        for a_ in range(block):  # diagonal block A_j (lower half)
            for b_ in range(a_ + 1):
                band[a_ - b_, c0 + b_] = Ah[a_, b_]
        if c1 < maxdim:  # coupling block B_j = T[c1:c1+block, c0:c1], upper triangular
            for a_ in range(block):
                for b_ in range(a_, block):
                    band[block + a_ - b_, c0 + b_] = Bh[a_, b_]
        Bprev = Bj
        used = c1
        if j + 1 >= next_check or j == nblk - 1:
            kk = min(k, used)
            theta, S = _band_ritz(band[:, :used], kk)
            res = np.linalg.norm(Bh @ S[used - block:used, :], axis=0)
            if np.all(res <= tol * max(abs(theta[-1]), 1e-300)):
                break
            # the check (a banded eigenvalue solve, O(basis^2)) outgrows the
            # blocks between checks: space the checks geometrically
            next_check = max(j + 1 + check_every, int(1.25 * (j + 1)))
    Y = Q[:, :used] @ torch.as_tensor(S, dtype=dt, device=dev)
    info = {"basis": used, "max_residual": float(res.max()), "theta_k": float(theta[-1])}
    return (torch.as_tensor(theta, dtype=dt, device=dev), Y.T.reshape(-1, 3, n),
            torch.as_tensor(res, dtype=dt, device=dev), info)


def traj_grad(state0, q, m, trap, dt, nsteps, checkpoint_every=50, eps2=0.0, prec="fp64"):
    """Mean-square displacement L = (1/n) sum_i |r_i(T) - r_i(0)|^2 after
    nsteps velocity-Verlet steps from state0 ((9, n) or (6, n) tensor; the
    accelerations are recomputed), and dL/d(wx, wy, wz) by the discrete
    adjoint, storing a checkpoint every `checkpoint_every` steps and
    recomputing each segment's positions in the backward pass.
    Returns (L, grad (3,), info)."""
    n = q.numel()
    dev = q.device
    st = torch.zeros(9, n, dtype=torch.float64, device=dev)
    st[:6] = state0[:6]
    S = [st[k] for k in range(9)]
    api.md_run(S, q, m, trap, 0.0, dt, 0, eps2=eps2, prec=prec, init_accel=True)
    r0 = st[:3].clone()
    ckpts = {0: st.clone()}
    done = 0
    while done < nsteps:
        k = min(checkpoint_every, nsteps - done)
        api.md_run(S, q, m, trap, done * dt, dt, k, eps2=eps2, prec=prec, init_accel=False)
        done += k
        if done < nsteps:
            ckpts[done] = st.clone()
    rT = st[:3].clone()
    L = float(((rT - r0) ** 2).sum()) / n
    lam = torch.zeros(9, n, dtype=torch.float64, device=dev)
    lam[:3] = 2.0 * (rT - r0) / n
    dldw = torch.zeros(3, dtype=torch.float64, device=dev)
    seg_starts = sorted(ckpts.keys())
    for s0 in reversed(seg_starts):
        s1 = min(s0 + checkpoint_every, nsteps)
        cur = ckpts[s0].clone()
        C = [cur[k] for k in range(9)]
        pos = []  # positions r_{s0+1} .. r_{s1}
        for step in range(s0, s1):
            api.md_step(C, q, m, trap, step * dt, dt, eps2=eps2, prec=prec)
            pos.append(cur[:3].clone())
        for step in range(s1 - 1, s0 - 1, -1):
            rp = pos[step - s0]
            api.md_adjoint_step(rp[0].contiguous(), rp[1].contiguous(), rp[2].contiguous(), q, m, trap, dt, lam,
                                dldw, eps2=eps2, prec=prec)
    api.md_adjoint_step(r0[0].contiguous(), r0[1].contiguous(), r0[2].contiguous(), q, m, trap, dt, lam, dldw,
                        eps2=eps2, prec=prec, final=True)
    return L, dldw, {"checkpoints": len(ckpts)}


def count_defects(x, y, z):
    """Kinks of a zigzag chain: ions sorted along z, the transverse
    displacement projected on the principal transverse axis, s_k = sign; a
    defect is a place where the zigzag order s_k = -s_{k+1} breaks
    (s_k = s_{k+1}).  Meaningful for quasi-one-dimensional crystals only."""
    x, y, z = (np.asarray(a, dtype=np.float64) for a in (x, y, z))
    order = np.argsort(z)
    P = np.stack([x[order] - x.mean(), y[order] - y.mean()])
    if P.shape[1] < 3:
        return 0
    w, V = np.linalg.eigh(P @ P.T)
    e = V[:, np.argmax(w)]
    s = np.sign(e @ P)
    s[s == 0] = 1
    return int(np.sum(s[1:] == s[:-1]))
