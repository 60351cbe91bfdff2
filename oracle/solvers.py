"""Textbook FP64 solvers of the oracle (test infrastructure only).

Written from the paper (Babich et al., SC11): CG and CG on the normal
equations (Section III-A), BiCGstab (Section III-A cites it; the paper's
baseline for GCR-DD, Section IX), the multi-shift CG for eq. (4) (Section
III-A; the method is cited there, not printed), minimal residual for the Schwarz blocks,
the additive Schwarz preconditioner (Section III-B, Section VIII-A) and its
multiplicative form over two block colours (Section III-B; Section X names
multiplicative and overlapping Schwarz as the next step), and
the GCR-DD solver of Algorithm 1 (Section VIII-A), all in FP64 with numpy
inner products <a,b> = sum conj(a) b. Every function takes the operator as a
callable.
"""
import numpy as np


def dot(a, b):
    return np.vdot(a, b)


def norm(a):
    return float(np.sqrt(np.vdot(a, a).real))


def cg(apply_A, b, tol=1e-10, maxiter=10000, x0=None):
    """Hestenes-Stiefel CG for a Hermitian positive-definite operator.
    Stops when ||b - A x|| (the recursively updated residual) <= tol ||b||.
    Returns (x, iterations, residual-norm history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    p = r.copy()
    rr = dot(r, r).real
    bn = norm(b)
    hist = [np.sqrt(rr)]
    it = 0
    while np.sqrt(rr) > tol * bn and it < maxiter:
        Ap = apply_A(p)
        alpha = rr / dot(p, Ap).real
        x += alpha * p
        r -= alpha * Ap
        rr_new = dot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
        hist.append(np.sqrt(rr))
    return x, it, hist


def bicgstab(apply_A, b, tol=1e-10, maxiter=10000, x0=None):
    """BiCGstab (van der Vorst) for a general non-singular A, shadow residual
    r^ = r_0:
        rho' = <r^, r>,  beta = (rho' / rho) (alpha / omega),
        p = r + beta (p - omega v),  v = A p,  alpha = rho' / <r^, v>,
        s = r - alpha v,  t = A s,  omega = <t, s> / <t, t>,
        x += alpha p + omega s,  r = s - omega t,
    starting from rho = alpha = omega = 1, p = v = 0. Stops when the
    recursively updated ||r|| (or ||s||, after the half step) <= tol ||b||.
    Returns (x, iterations, residual-norm history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    rh = r.copy()
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    rho = alpha = omega = 1.0
    bn = norm(b)
    hist = [norm(r)]
    it = 0
    while hist[-1] > tol * bn and it < maxiter:
        rho_new = dot(rh, r)
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply_A(p)
        alpha = rho_new / dot(rh, v)
        s_ = r - alpha * v
        it += 1
        if norm(s_) <= tol * bn:
            x = x + alpha * p
            hist.append(norm(s_))
            break
        t = apply_A(s_)
        omega = dot(t, s_) / dot(t, t)
        x = x + alpha * p + omega * s_
        r = s_ - omega * t
        rho = rho_new
        hist.append(norm(r))
    return x, it, hist


def multishift_cg(apply_A, b, shifts, tol=1e-10, maxiter=10000):
    """All solutions of (A + s_i) x_i = b (eq. (4)) from the one Krylov space
    of CG on A (A Hermitian positive definite, A + s_i too). The residual of
    shifted system i stays collinear with the base residual, r_i = z_i r, and
    the CG recurrences of the base fix every z_i:
        z_{k+1} = z_k z_{k-1} a_{k-1} /
                  (a_k b_{k-1} (z_{k-1} - z_k) + z_{k-1} a_{k-1} (1 + s a_k)),
        a^s_k = a_k z_{k+1} / z_k,   b^s_k = b_k (z_{k+1} / z_k)^2,
        x^s += a^s_k p^s,   p^s = z_{k+1} r_{k+1} + b^s_k p^s,
    with z_0 = z_{-1} = 1, a_{-1} = 1, b_{-1} = 0. A shift stops being updated
    once |z| ||r|| <= tol ||b||; the iteration ends when all have.
    Returns (list of x_i, iterations, list of |z_i| ||r|| / ||b|| at each
    shift's last update)."""
    shifts = [float(s_) for s_ in shifts]
    ns = len(shifts)
    r = b.copy()
    p = b.copy()
    xs = [np.zeros_like(b) for _ in range(ns)]
    ps = [b.copy() for _ in range(ns)]
    z = [1.0] * ns        # z_k
    z_prev = [1.0] * ns   # z_{k-1}
    a_prev, b_prev = 1.0, 0.0
    rr = dot(r, r).real
    bn = norm(b)
    active = [True] * ns
    res = [1.0] * ns
    it = 0
    while any(active) and it < maxiter:
        Ap = apply_A(p)
        a = rr / dot(p, Ap).real
        r = r - a * Ap
        rr_new = dot(r, r).real
        bk = rr_new / rr
        for i in range(ns):
            if not active[i]:
                continue
            s_ = shifts[i]
            z_next = z[i] * z_prev[i] * a_prev / (a * b_prev * (z_prev[i] - z[i]) + z_prev[i] * a_prev * (1.0 + s_ * a))
            a_s = a * z_next / z[i]
            b_s = bk * (z_next / z[i]) ** 2
            xs[i] = xs[i] + a_s * ps[i]
            ps[i] = z_next * r + b_s * ps[i]
            z_prev[i], z[i] = z[i], z_next
        p = r + bk * p
        a_prev, b_prev = a, bk
        rr = rr_new
        it += 1
        for i in range(ns):
            if active[i]:
                res[i] = abs(z[i]) * np.sqrt(rr) / bn
                if res[i] <= tol:
                    active[i] = False
    return xs, it, res


def cgne(apply_A, apply_Adag, b, tol=1e-10, maxiter=10000, x0=None):
    """CG on the normal equations A A^+ y = b, x = A^+ y (Craig's method).
    r = b - A x is the true residual of A x = b in exact arithmetic.
    Returns (x, iterations, residual-norm history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    p = apply_Adag(r)
    rr = dot(r, r).real
    bn = norm(b)
    hist = [np.sqrt(rr)]
    it = 0
    while np.sqrt(rr) > tol * bn and it < maxiter:
        alpha = rr / dot(p, p).real
        x += alpha * p
        r -= alpha * apply_A(p)
        rr_new = dot(r, r).real
        p = apply_Adag(r) + (rr_new / rr) * p
        rr = rr_new
        it += 1
        hist.append(np.sqrt(rr))
    return x, it, hist


def mr_blocks(apply_A, b, nsteps, labels=None, site_axes=4, omega=1.0):
    """Minimal-residual iteration started from x = 0, r = b, run independently on
    every Dirichlet block: inner products are summed over one block only
    (domain-restricted reductions, Section VIII-A). labels: integer block id per
    site (natural grid) or None for one block. Each step:
        q = A r ; alpha = omega <q,r>/<q,q> ; x += alpha r ; r -= alpha q,
    omega the over-relaxation factor (1: plain MR; the paper gives none).
    """
    x = np.zeros_like(b)
    r = b.copy()
    if labels is None:
        for _ in range(nsteps):
            q = apply_A(r)
            qq = dot(q, q).real
            if qq == 0.0:
                break
            alpha = omega * dot(q, r) / qq
            x += alpha * r
            r -= alpha * q
        return x
    lab = labels.reshape(-1)
    nb = int(lab.max()) + 1
    inner = int(np.prod(b.shape[site_axes:]))
    for _ in range(nsteps):
        q = apply_A(r)
        qf = q.reshape(-1, inner)
        rf = r.reshape(-1, inner)
        qr = np.bincount(lab, weights=np.sum(np.conj(qf) * rf, axis=1).real, minlength=nb) \
            + 1j * np.bincount(lab, weights=np.sum(np.conj(qf) * rf, axis=1).imag, minlength=nb)
        qq = np.bincount(lab, weights=np.sum(np.abs(qf) ** 2, axis=1), minlength=nb)
        alpha = omega * np.where(qq > 0, qr / np.where(qq > 0, qq, 1.0), 0.0)
        a_site = alpha[labels].reshape(labels.shape + (1,) * (b.ndim - site_axes))
        x += a_site * r
        r -= a_site * q
    return x


def schwarz(op, r, block, nsteps, omega=1.0):
    """Non-overlapping additive Schwarz preconditioner (block Jacobi,
    Section III-B): on every block B of size `block`, nsteps of MR on the
    Dirichlet-cut even-odd operator Mhat_B with block-restricted inner products.
    op is an oracle.WilsonClover; r lives on even sites."""
    from . import block_labels
    labels = block_labels(op.dims, block)
    return mr_blocks(lambda v: op.schur(v, block=block), r, nsteps, labels, omega=omega)


def block_colour(dims, block):
    """Colour of every site's Dirichlet block: the sum of the block's
    coordinates modulo 2 (a checkerboard of blocks, so that two blocks of one
    colour never share a face)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    bx, by, bz, bt = (int(b) for b in block)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    return (x // bx + y // by + z // bz + t // bt) % 2


def sap(op, r, block, nsteps, ncycles, omega=1.0):
    """Multiplicative Schwarz (the Schwarz alternating procedure) on the
    Dirichlet blocks of `block`, coloured as a checkerboard (block_colour).
    Starting from x = 0, each cycle visits colour 0 then colour 1; a visit
    takes the current residual r - Mhat x of the whole even-odd system,
    keeps it on the blocks of that colour, runs nsteps of block MR on the
    Dirichlet-cut Mhat_B there (as the additive preconditioner does on every
    block) and adds the result to x. Blocks of the other colour see the
    update through the next residual. op is an oracle.WilsonClover; r lives
    on even sites."""
    from . import block_labels
    labels = block_labels(op.dims, block)
    colour = block_colour(op.dims, block)
    x = np.zeros_like(r)
    for _ in range(ncycles):
        for c in (0, 1):
            res = r - op.schur(x)
            res = np.where(((colour == c) & op.even)[..., None, None], res, 0)
            x = x + mr_blocks(lambda v: op.schur(v, block=block), res, nsteps, labels, omega=omega)
    return x


def gcr(apply_M, precond, b, tol=1e-10, kmax=16, delta=1e-3, maxiter=10000, x0=None, record=None):
    """GCR with restarts, Algorithm 1, entirely in FP64.

    Readings: the stopping tests are relative to ||b||; the normalisation
    step divides the orthogonalised z_k by gamma_k; the restart residual is
    r0 = b - M x. Orthogonalisation is modified Gram-Schmidt as printed.
    precond(r) returns K r (None: K = 1).
    record: optional dict that receives per-step diagnostics.
    Returns (x, total Krylov steps, restarts, list of true residual norms at restarts).
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = norm(b)
    r0 = b - apply_M(x)
    rhat = r0.copy()
    r0n = norm(r0)
    true_hist = [r0n]
    p, z, alpha, gamma = [], [], [], []
    beta = {}
    k = 0
    steps = 0
    restarts = 0
    while r0n > tol * bn and steps < maxiter:
        pk = precond(rhat) if precond is not None else rhat.copy()
        zk = apply_M(pk)
        for i in range(k):
            beta[(i, k)] = dot(z[i], zk)
            zk = zk - beta[(i, k)] * z[i]
        g = norm(zk)
        zk = zk / g
        a = dot(zk, rhat)
        rhat = rhat - a * zk
        p.append(pk)
        z.append(zk)
        gamma.append(g)
        alpha.append(a)
        k += 1
        steps += 1
        rn = norm(rhat)
        if record is not None:
            record.setdefault("rhat", []).append(rn)
            record.setdefault("z", []).append(zk)
            record.setdefault("rvec", []).append(rhat.copy())
        if k == kmax or rn / r0n < delta or rn < tol * bn or steps >= maxiter:
            chi = [0j] * k
            for l in range(k - 1, -1, -1):
                s = alpha[l]
                for i in range(l + 1, k):
                    s -= beta[(l, i)] * chi[i]
                chi[l] = s / gamma[l]
            xhat = np.zeros_like(b)
            for i in range(k):
                xhat += chi[i] * p[i]
            if record is not None:
                record.setdefault("restart_check", []).append((apply_M(xhat), r0 - rhat))
            x += xhat
            r0 = b - apply_M(x)
            r0n = norm(r0)
            true_hist.append(r0n)
            rhat = r0.copy()
            p, z, alpha, gamma, beta = [], [], [], [], {}
            k = 0
            restarts += 1
    return x, steps, restarts, true_hist
