"""Pins of the RBF level-set oracle (Eqs. 2, 3 and the renormalisation that
follows them) and of its Adam update, against geometry, textbook norms,
invariants of the shift, complex-step derivatives and the closed form of
Adam's moving averages."""
import numpy as np
import pytest

from oracle import rbf

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def random_rbfs(rng, n, nx, ny):
    xc = rng.uniform(0, nx - 1, n)
    yc = rng.uniform(0, ny - 1, n)
    s = rng.uniform(-4.0, 6.0, n)
    return s, (xc, yc)


def test_single_rbf_is_a_cone_with_a_circular_zero_set():
    """One RBF: the p-norm of one non-negative base is the base, so Phi is the
    cone itself whatever the shift: apex s - c on its centre node, zero set on
    the circle of radius sqrt(s^2 - c^2) about the centre (an off-diagonal
    centre on a non-square grid, so swapped axes fail), slope -> -1 far out."""
    nx, ny, c, s = 48, 40, 1.5, 9.0
    xc, yc = 31.0, 12.0
    design = np.ones((ny, nx))
    phi, dphi, _ = rbf.pnorm_levelset(np.array([s]), (np.array([xc]), np.array([yc])), c, 90.0, design,
                                      normalize=False)
    assert dphi > 0
    assert phi[12, 31] == pytest.approx(s - c, abs=1e-12)
    assert phi.max() == pytest.approx(s - c, abs=1e-12)
    R = np.sqrt(s * s - c * c)
    for iy in range(ny):
        for ix in range(nx):
            r = np.hypot(ix - xc, iy - yc)
            if abs(r - R) > 1e-6:
                assert (phi[iy, ix] > 0) == (r < R), (ix, iy)
    row = phi[12, :]
    steps = np.diff(row[:12])      # x from 0 to 11: at least 20 nodes left of the centre, rising by ~1 per node
    assert np.all(steps > 0.99) and np.all(steps < 1.0)


def test_pnorm_reduces_to_sum_and_euclidean_norm():
    """p = 1: the 1-norm of non-negative bases is their sum; p = 2: their
    Euclidean length (numpy.linalg.norm over the RBF axis)."""
    rng = np.random.default_rng(0)
    nx, ny, n, c = 23, 17, 9, 1.0
    s, ctr = random_rbfs(rng, n, nx, ny)
    design = np.ones((ny, nx))
    g = np.stack([[[s[i] - np.sqrt((ix - ctr[0][i]) ** 2 + (iy - ctr[1][i]) ** 2 + c * c)
                    for ix in range(nx)] for iy in range(ny)] for i in range(n)])
    d = abs(g.min())
    phi1, _, _ = rbf.pnorm_levelset(s, ctr, c, 1.0, design, normalize=False)
    np.testing.assert_allclose(phi1, (g + d).sum(axis=0) - d, rtol=1e-12, atol=1e-11)
    phi2, _, _ = rbf.pnorm_levelset(s, ctr, c, 2.0, design, normalize=False)
    np.testing.assert_allclose(phi2, np.linalg.norm(g + d, axis=0) - d, rtol=1e-12, atol=1e-11)


def test_pnorm_brackets_the_maximum_rbf():
    """The p-norm lies between the max-norm and n^(1/p) times it, so
    max_i g_i <= Phi <= n^(1/p) (max_i g_i + dphi) - dphi, node by node,
    against a brute-force maximum over the RBFs; at p = 90 the bracket is
    tight (n^(1/90) - 1 < 0.05 for n <= 80)."""
    rng = np.random.default_rng(1)
    nx, ny, n, c, p = 30, 26, 80, 2.0, 90.0
    s, ctr = random_rbfs(rng, n, nx, ny)
    design = np.ones((ny, nx))
    phi, dphi, _ = rbf.pnorm_levelset(s, ctr, c, p, design, normalize=False)
    for iy in range(0, ny, 3):
        for ix in range(0, nx, 3):
            gmax = max(s[i] - np.sqrt((ix - ctr[0][i]) ** 2 + (iy - ctr[1][i]) ** 2 + c * c) for i in range(n))
            assert gmax - 1e-10 <= phi[iy, ix] <= n ** (1 / p) * (gmax + dphi) - dphi + 1e-10
            assert phi[iy, ix] - gmax <= 0.05 * (gmax + dphi)


def test_shift_is_the_smallest_rbf_on_the_design_region():
    """dphi = |min over RBFs and design nodes of g_i|, by brute force over a
    design region that excludes where the global minimum lies; every base
    g_i + dphi on the design region is then non-negative."""
    rng = np.random.default_rng(2)
    nx, ny, n, c = 20, 16, 7, 1.0
    s, ctr = random_rbfs(rng, n, nx, ny)
    design = np.zeros((ny, nx))
    design[4:12, 5:15] = 1
    best = np.inf
    best_all = np.inf
    for i in range(n):
        for iy in range(ny):
            for ix in range(nx):
                v = s[i] - np.sqrt((ix - ctr[0][i]) ** 2 + (iy - ctr[1][i]) ** 2 + c * c)
                best_all = min(best_all, v)
                if design[iy, ix]:
                    best = min(best, v)
    assert best_all < best
    g = rbf.cones(s, ctr, c, nx, ny)
    assert rbf.shift(g, design) == pytest.approx(abs(best), abs=1e-13)
    assert (g[:, design.astype(bool)] + rbf.shift(g, design)).min() >= 0


def test_common_offset_of_amplitudes_shifts_phi():
    """Adding k to every amplitude raises every cone by k; while the smallest
    cone stays negative the shift absorbs it, the bases stay the same, and
    Phi rises by exactly k (a sign slip in the shift gives -k)."""
    rng = np.random.default_rng(3)
    nx, ny, n, c = 25, 21, 12, 1.0
    s, ctr = random_rbfs(rng, n, nx, ny)
    design = np.ones((ny, nx))
    phi0, d0, _ = rbf.pnorm_levelset(s, ctr, c, 90.0, design, normalize=False)
    k = 0.37
    phi1, d1, _ = rbf.pnorm_levelset(s + k, ctr, c, 90.0, design, normalize=False)
    assert d1 == pytest.approx(d0 - k, abs=1e-12)
    np.testing.assert_allclose(phi1 - phi0, k, atol=1e-11)


def test_order_of_rbfs_does_not_matter_and_renormalisation_keeps_the_boundary():
    rng = np.random.default_rng(4)
    nx, ny, n, c = 27, 19, 15, 1.3
    s, ctr = random_rbfs(rng, n, nx, ny)
    design = np.zeros((ny, nx))
    design[2:17, 3:24] = 1
    D = design.astype(bool)
    phi, _, scale = rbf.pnorm_levelset(s, ctr, c, 90.0, design)
    perm = rng.permutation(n)
    phip, _, _ = rbf.pnorm_levelset(s[perm], (ctr[0][perm], ctr[1][perm]), c, 90.0, design)
    np.testing.assert_allclose(phip, phi, rtol=1e-13, atol=1e-13)
    raw, _, _ = rbf.pnorm_levelset(s, ctr, c, 90.0, design, normalize=False)
    assert np.abs(phi[D]).max() == pytest.approx(1.0, abs=1e-15)
    assert np.array_equal(np.sign(phi[D]), np.sign(raw[D]))
    assert scale > 0


@pytest.mark.parametrize("normalize", [True, False])
def test_vjp_matches_complex_step(normalize):
    """dJ/ds by the closed-form VJP against the complex-step derivative of the
    map with the shift and the scale held at their values (they are chosen from
    the current amplitudes, not differentiated)."""
    rng = np.random.default_rng(5)
    nx, ny, n, c, p = 22, 18, 10, 1.0, 90.0
    s, ctr = random_rbfs(rng, n, nx, ny)
    design = np.zeros((ny, nx))
    design[1:16, 2:20] = 1
    phi, dphi, scale = rbf.pnorm_levelset(s, ctr, c, p, design, normalize=normalize)
    w = rng.standard_normal((ny, nx)) * design
    got = rbf.pnorm_levelset_vjp(s, ctr, c, p, design, w, dphi, scale)
    h = 1e-30
    want = np.empty(n)
    for i in range(n):
        sc = s.astype(complex)
        sc[i] += 1j * h
        ph, _, _ = rbf.pnorm_levelset(sc, ctr, c, p, design, frozen=(dphi, scale))
        want[i] = np.sum(w * ph.imag) / h
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12 * np.abs(want).max())


def test_adam_first_step_is_lr_times_sign():
    """With bias correction the first step is lr * g / (|g| + eps): a step of
    lr against the sign of every component (|g| >> eps)."""
    rng = np.random.default_rng(6)
    s = rng.standard_normal(50)
    g = rng.choice([-1.0, 1.0], 50) * np.logspace(-2, 3, 50)
    s1, _, _ = rbf.adam_step(s, g, np.zeros(50), np.zeros(50), 1, lr=0.01)
    np.testing.assert_allclose(s - s1, 0.01 * np.sign(g), rtol=1e-5)


def test_adam_constant_gradient_moves_by_lr_each_step():
    s = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -7.0, 1e-2])
    m = v = np.zeros(3)
    for t in range(1, 30):
        s_new, m, v = rbf.adam_step(s, g, m, v, t, lr=0.05)
        np.testing.assert_allclose(s - s_new, 0.05 * np.sign(g), rtol=1e-5)
        s = s_new


def test_adam_moments_match_their_closed_form():
    """m_t = (1 - b1) sum_k b1^(t-k) g_k and v_t likewise (the unrolled moving
    averages); the step then uses m_t / (1 - b1^t) and v_t / (1 - b2^t)."""
    rng = np.random.default_rng(7)
    T, n, lr, b1, b2, eps = 6, 8, 3e-3, 0.9, 0.999, 1e-8
    gs = rng.standard_normal((T, n))
    s = rng.standard_normal(n)
    m = v = np.zeros(n)
    cur = s.copy()
    for t in range(1, T + 1):
        prev = cur
        cur, m, v = rbf.adam_step(cur, gs[t - 1], m, v, t, lr=lr, beta1=b1, beta2=b2, eps=eps)
        mt = sum((1 - b1) * b1 ** (t - k) * gs[k - 1] for k in range(1, t + 1))
        vt = sum((1 - b2) * b2 ** (t - k) * gs[k - 1] ** 2 for k in range(1, t + 1))
        np.testing.assert_allclose(m, mt, rtol=1e-13)
        np.testing.assert_allclose(v, vt, rtol=1e-13)
        step = lr * (mt / (1 - b1 ** t)) / (np.sqrt(vt / (1 - b2 ** t)) + eps)
        np.testing.assert_allclose(prev - cur, step, rtol=1e-12)


def test_adam_descends_an_ill_conditioned_quadratic():
    A = np.diag([1.0, 100.0, 1e4])
    x = np.array([3.0, -2.0, 1.0])
    m = v = np.zeros(3)
    lr = 0.05
    for t in range(1, 4001):
        if t % 1000 == 0:
            lr *= 0.1
        x, m, v = rbf.adam_step(x, A @ x, m, v, t, lr=lr)
    assert np.abs(x).max() < 1e-2


def test_vjp_at_the_kink_takes_the_zero_subgradient():
    """One cone on a design region: the node where it is smallest has the base
    0 and a p-norm of 0 (a kink); that node adds nothing, and every other node
    adds scale * dJ/dphi (one base: (b / S)^(p-1) = 1)."""
    s, ctr, c = np.array([2.0]), (np.array([1.0]), np.array([1.0])), 1.0
    design = np.ones((5, 7))
    phi, dphi, scale = rbf.pnorm_levelset(s, ctr, c, 90.0, design)
    w = np.ones((5, 7))
    g = rbf.cones(s, ctr, c, 7, 5)[0]
    kink = g == g.min()
    assert kink.sum() == 1
    got = rbf.pnorm_levelset_vjp(s, ctr, c, 90.0, design, w, dphi, scale)
    assert got[0] == pytest.approx(scale * (w.size - 1), rel=1e-14)
