"""Pins of the CPU oracle's lattice Boltzmann part against facts the paper
and the mathematics fix (no GPU).  Each test names what it pins."""
import numpy as np
import pytest

from paper_1601_02708_amd import inputs


# ----------------------------------------------------------------------------
# D2Q9 constants and the equilibrium (Sec. 4.1, eq. LBM_feq)
# ----------------------------------------------------------------------------

def test_d2q9_moments(orc):
    ex, ey, w, opp = orc.d2q9()
    e = np.stack([ex, ey], 1).astype(float)
    assert np.isclose(w.sum(), 1.0, atol=1e-15)
    assert np.allclose(w @ e, 0.0, atol=1e-16)
    # second moment c_s^2 I with c_s^2 = 1/3 (Sec. 4.1: c_s = dx / (sqrt(3) dt))
    assert np.allclose(np.einsum("i,ia,ib->ab", w, e, e), np.eye(2) / 3.0, atol=1e-16)
    # fourth-moment isotropy fixes the textbook weights 4/9, 1/9, 1/36
    assert np.isclose((w * e[:, 0] ** 4).sum(), 1.0 / 3.0)
    assert np.isclose((w * e[:, 0] ** 2 * e[:, 1] ** 2).sum(), 1.0 / 9.0)
    assert np.all(e[opp] == -e)
    assert sorted(map(tuple, e.astype(int))) == sorted(
        [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])


def test_equilibrium_moments(orc):
    """Zeroth, first and second moments of the equilibrium: u, u v and
    u (c_s^2 I + v v).  The mass moment pins the reading of the quadratic
    term as -v.v/(2 c_s^2)."""
    ex, ey, w, _ = orc.d2q9()
    e = np.stack([ex, ey], 1).astype(float)
    rng = np.random.default_rng(1)
    for _ in range(20):
        u = rng.uniform(0.1, 2.0)
        v = rng.uniform(-0.1, 0.1, 2)
        f = orc.feq(u, v[0], v[1])
        assert abs(f.sum() - u) <= 1e-15 * u * 4
        assert np.allclose(f @ e, u * v, atol=1e-15)
        P = np.einsum("i,ia,ib->ab", f, e, e)
        assert np.allclose(P, u * (np.eye(2) / 3.0 + np.outer(v, v)), atol=1e-15)


def _lattice(orc, N, tau, v=(0.0, 0.0), solid=None, k=0.0, px=True, py=True, bc_kind=None, clamp=False):
    vx = np.full((N, N), v[0])
    vy = np.full((N, N), v[1])
    if solid is not None:
        vx[solid != 0] = 0.0
        vy[solid != 0] = 0.0
    return orc.Lattice(N, tau, vx, vy, solid=solid, k=k, periodic_x=px, periodic_y=py, bc_kind=bc_kind,
                       clamp=clamp)


def test_collision_mass_and_reaction(orc):
    """Summing the collision over i: sum f* = (1 - k) sum f (per node)."""
    N = 8
    rng = np.random.default_rng(2)
    k = rng.uniform(0, 1e-2, (N, N))
    lat = orc.Lattice(N, 0.7, rng.uniform(-.05, .05, (N, N)), rng.uniform(-.05, .05, (N, N)), k=k)
    f = rng.uniform(0.1, 1.0, (9, N, N))
    fs = lat.collide(f)
    assert np.allclose(fs.sum(0), (1 - k) * f.sum(0), rtol=1e-14)
    # concentration readout inverts it
    assert np.allclose(lat.concentration(fs), f.sum(0), rtol=1e-14)


def test_collision_relaxes_to_equilibrium(orc):
    """tau = 1 maps any population to the equilibrium of its own moment."""
    N = 4
    rng = np.random.default_rng(3)
    vx = rng.uniform(-.05, .05, (N, N))
    vy = rng.uniform(-.05, .05, (N, N))
    lat = orc.Lattice(N, 1.0, vx, vy)
    f = rng.uniform(0.1, 1.0, (9, N, N))
    fs = lat.collide(f)
    for j in range(N):
        for i in range(N):
            assert np.allclose(fs[:, j, i], orc.feq(f[:, j, i].sum(), vx[j, i], vy[j, i]), rtol=1e-14)


# ----------------------------------------------------------------------------
# streaming / bounce-back invariants on periodic boxes
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("tau", [0.53, 1.2])
def test_periodic_mass_conservation_with_solids(orc, tau):
    """P1: BGK collision, periodic streaming and halfway bounce-back conserve
    total mass exactly (k = 0)."""
    N = 48
    pack = inputs.random_disks(N, 0.7, seed=5, r_min=3, r_max=7, margin=2)
    lat = _lattice(orc, N, tau, v=(0.03, -0.02), solid=pack.solid)
    fs = inputs.random_populations(N, 7)
    fs[:, pack.solid != 0] = 0.0
    m0 = fs.sum()
    for _ in range(2000):
        fs, _inf = lat.substep(fs)
    assert abs(fs.sum() - m0) <= 1e-13 * m0


def test_streaming_is_a_shift(orc):
    """Pull streaming on a periodic box moves population i by +e_i."""
    N = 6
    ex, ey, _, _ = orc.d2q9()
    lat = _lattice(orc, N, 1.0)
    fs = inputs.random_populations(N, 11)
    f, unk = lat.stream(fs)
    assert not unk.any()
    for q in range(9):
        assert np.array_equal(f[q], np.roll(np.roll(fs[q], ey[q], axis=0), ex[q], axis=1))


def test_bounce_back_single_link(orc):
    """Halfway bounce-back: a population sent into a solid neighbour comes
    back reversed to the sender on the next step."""
    N = 5
    solid = np.zeros((N, N), np.uint8)
    solid[2, 3] = 1                     # node (i=3, j=2)
    ex, ey, _, opp = orc.d2q9()
    lat = _lattice(orc, N, 1.0, solid=solid)
    fs = inputs.random_populations(N, 12)
    f, _ = lat.stream(fs)
    # node (i=2, j=2): its source along e_1 = (1,0) is (1,2) (fluid); along
    # e_3 = (-1,0) the source is (3,2), which is solid -> f_3 = f*_1(2,2)
    assert f[3, 2, 2] == fs[1, 2, 2]
    assert f[1, 2, 2] == fs[1, 2, 1]
    # solid node receives nothing
    assert np.all(f[:, 2, 3] == 0)


def test_uniform_decay_with_reaction(orc):
    """P2: uniform concentration with uniform velocity on a periodic box
    decays as u_n = u_0 (1 - k)^n at every node."""
    N, k, n = 16, 1e-3, 300
    lat = _lattice(orc, N, 0.56, v=(0.04, 0.02), k=k)
    fs = lat.init(np.full((N, N), 2.0))
    for _ in range(n):
        fs, _ = lat.substep(fs)
    u = lat.concentration(fs)
    assert np.allclose(u, 2.0 * (1 - k) ** n, rtol=1e-13)


def test_h_theorem_periodic(orc):
    """P6: with v = 0 and tau >= 1 the H function of eq. (BH) does not
    increase (streaming permutes populations; the collision is a convex
    combination with the H-minimising equilibrium)."""
    N = 24
    lat = _lattice(orc, N, 1.3)
    fs = inputs.random_populations(N, 13, lo=0.01, hi=1.0)
    H = [lat.h_function(fs)]
    for _ in range(200):
        fs, _ = lat.substep(fs)
        H.append(lat.h_function(fs))
    H = np.asarray(H)
    assert np.all(np.diff(H) <= 1e-14 * np.abs(H[:-1]))
    assert H[-1] < H[0]


def test_positivity_tau_ge_one(orc):
    """Sec. 4.1, eq. (NN_Cond): with 1 - 1/tau >= 0 populations stay
    non-negative, including at maxent Dirichlet walls when the closure keeps
    f >= 0 (clamped variant; the data here make some nodes infeasible)."""
    N = 20
    lat = _lattice(orc, N, 1.05, v=(0.02, 0.01), px=False, py=False, clamp=True)
    fs = inputs.random_populations(N, 14, lo=0.0, hi=1.0)
    bc = np.random.default_rng(15).uniform(0.0, 3.0, 4 * (N - 1))
    for _ in range(300):
        fs, _ = lat.substep(fs, bc)
        assert fs.min() >= 0.0


# ----------------------------------------------------------------------------
# boundary closures (Sec. 4.1.1)
# ----------------------------------------------------------------------------

def test_linear_profile_fixed_point(orc):
    """P3: between Dirichlet walls at i = 0 and i = N-1 (periodic in y,
    v = 0) the linear profile u = A + c x is reproduced exactly by the
    post-collision state f*_i = w_i (u - (tau - 1) c e_ix); the maxent
    closure fills the wall unknowns with exactly these values."""
    N, tau, A, c = 12, 0.8, 1.0, 0.05
    ex, ey, w, _ = orc.d2q9()
    lat = _lattice(orc, N, tau, px=False, py=True)
    x = np.arange(N, dtype=float)[None, :].repeat(N, 0)
    u = A + c * x
    fs = np.stack([w[q] * (u - (tau - 1) * c * ex[q]) for q in range(9)])
    ii, jj = orc.perimeter_nodes(N)
    bc = A + c * ii.astype(float)
    out, inf = lat.substep(fs, bc)
    assert inf == 0
    assert np.allclose(out, fs, rtol=1e-13, atol=1e-15)


def test_linear_profile_converges_from_rest(orc):
    """P3 (transient): from u = 0 the lattice relaxes to the linear
    profile between the two Dirichlet walls."""
    N, tau = 10, 0.9
    lat = _lattice(orc, N, tau, px=False, py=True)
    fs = np.zeros((9, N, N))
    ii, jj = orc.perimeter_nodes(N)
    bc = np.where(ii == 0, 1.0, np.where(ii == N - 1, 3.0, 0.0))
    for _ in range(4000):
        fs, _ = lat.substep(fs, bc)
    u = lat.concentration(fs)
    expect = 1.0 + 2.0 * np.arange(N) / (N - 1)
    assert np.allclose(u, expect[None, :], rtol=1e-12)


def _h(f, w):
    return float(np.sum(f * np.log(f / w)))


@pytest.mark.parametrize("unknown", [0b100100010, 0b101100110, 0b000010000 | 0b010000000 | 0b100000000])
def test_maxent_dirichlet(orc, unknown):
    """P7 Dirichlet: the closure is the minimiser of H over the unknowns
    subject to sum f = u^p (checked against a generic constrained optimiser),
    non-negative, and its KKT stationarity log(f_i/w_i) = const holds."""
    from scipy.optimize import minimize
    _, _, w, _ = orc.d2q9()
    rng = np.random.default_rng(unknown)
    U = [q for q in range(9) if unknown >> q & 1]
    f = rng.uniform(0.05, 0.3, 9)
    known = sum(f[q] for q in range(9) if q not in U)
    up = known + rng.uniform(0.1, 1.0)
    out, inf = orc.maxent_dirichlet(f, unknown, up)
    assert inf == 0
    assert abs(out.sum() - up) <= 1e-13 * up
    assert np.all(out >= 0)
    lg = np.log(out[U] / w[U])
    assert np.ptp(lg) < 1e-13
    # independent: minimise H numerically
    res = minimize(lambda z: _h(z, w[U]), x0=np.full(len(U), (up - known) / len(U)),
                   constraints=[{"type": "eq", "fun": lambda z: z.sum() - (up - known)}],
                   bounds=[(1e-14, None)] * len(U), method="SLSQP",
                   options={"ftol": 1e-15, "maxiter": 500})
    assert np.allclose(res.x, out[U], rtol=1e-6)
    # known populations are untouched
    for q in range(9):
        if q not in U:
            assert out[q] == f[q]
    # infeasible: u^p below the known mass.  As printed the closure still
    # meets sum f = u^p (negative unknowns); the clamped variant keeps
    # f >= 0 and sets the unknowns to zero.  Both report the node.
    out2, inf2 = orc.maxent_dirichlet(f, unknown, known - 0.01)
    assert inf2 == 1 and abs(out2.sum() - (known - 0.01)) < 1e-14 and np.all(out2[U] < 0)
    out3, inf3 = orc.maxent_dirichlet(f, unknown, known - 0.01, clamp=True)
    assert inf3 == 1 and np.all(out3[U] == 0.0)


@pytest.mark.parametrize("corner", [False, True])
def test_maxent_neumann(orc, corner):
    """P7 Neumann, eq. (LBM_Neu): the flux constraint holds, the unknowns of
    M- are the H minimiser under that constraint (generic optimiser), KKT
    log(f_i/w_i) + 1 + gamma e_i.n = 0 with one gamma; at a corner the two
    tangential unknowns are bounced back from the node's own f*."""
    from scipy.optimize import minimize
    ex, ey, w, opp = orc.d2q9()
    rng = np.random.default_rng(21 + corner)
    if corner:   # bottom-left corner, outward normal (-1,-1)/sqrt(2)
        sx, sy = -1, -1
        unknown = sum(1 << q for q in range(9) if ex[q] == 1 or ey[q] == 1)
    else:        # left edge, outward normal (-1, 0)
        sx, sy = -1, 0
        unknown = sum(1 << q for q in range(9) if ex[q] == 1)
    n = np.array([sx, sy], float) / np.hypot(sx, sy)
    a = ex * n[0] + ey * n[1]
    Mm = [q for q in range(9) if (unknown >> q & 1) and a[q] < -1e-12]
    T = [q for q in range(9) if (unknown >> q & 1) and abs(a[q]) < 1e-12]
    f = rng.uniform(0.05, 0.3, 9)
    fstar_self = rng.uniform(0.05, 0.3, 9)
    qp = -0.05
    out, inf = orc.maxent_neumann(f, unknown, sx, sy, qp, fstar_self)
    assert inf == 0
    for q in T:
        assert out[q] == fstar_self[opp[q]]
    assert abs(np.dot(out, a) - qp) <= 1e-13
    lg = np.log(out[Mm] / w[Mm]) + 1.0
    gam = -lg / a[Mm]
    assert np.ptp(gam) < 1e-12
    rhs = qp - sum(a[q] * out[q] for q in range(9) if q not in Mm)
    res = minimize(lambda z: _h(z, w[Mm]), x0=np.full(len(Mm), 0.1),
                   constraints=[{"type": "eq", "fun": lambda z: np.dot(z, a[Mm]) - rhs}],
                   bounds=[(1e-14, None)] * len(Mm), method="SLSQP",
                   options={"ftol": 1e-15, "maxiter": 500})
    # The Lagrangian form f = w exp(-1 - gamma a) fixes the scale of the
    # optimum only through the constraint; SLSQP finds the same point.
    assert np.allclose(res.x, out[Mm], rtol=1e-5)
    # infeasible: the required inflow flux cannot be met by f >= 0
    out2, inf2 = orc.maxent_neumann(f, unknown, sx, sy, 10.0, fstar_self)
    assert inf2 == 1 and np.all(out2[Mm] == 0.0)


def test_neumann_zero_flux_flat_wall(orc):
    """Flat zero-flux wall: unknowns are proportional to w_i and carry the
    same normal flux as the known outgoing populations."""
    ex, ey, w, _ = orc.d2q9()
    unknown = sum(1 << q for q in range(9) if ey[q] == -1)   # top edge, n = (0, 1)
    f = np.random.default_rng(31).uniform(0.05, 0.3, 9)
    out, inf = orc.maxent_neumann(f, unknown, 0, 1, 0.0, f)
    U = [q for q in range(9) if ey[q] == -1]
    O = [q for q in range(9) if ey[q] == 1]
    assert inf == 0
    assert np.isclose(out[U].sum(), f[O].sum(), rtol=1e-14)
    assert np.allclose(out[U] / w[U], out[U[0]] / w[U[0]], rtol=1e-14)


def test_gaussian_pulse_second_order(orc):
    """P4: an advected, spreading Gaussian on a periodic unit square against
    the analytic ADE solution (sigma_t^2 = sigma_0^2 + 2 D t, centre moving
    with v, periodic images summed); diffusive refinement (tau fixed) gives
    second-order convergence."""
    tau, Dp, vp, s0, x0 = 0.8, 0.01, (0.1, 0.05), 0.1, (0.45, 0.5)
    errs = []
    for N in (32, 64, 128):
        Dl = (tau - 0.5) / 3.0
        h = 1.0 / N
        dt = Dl * h * h / Dp
        steps = 100 * (N // 32) ** 2
        T = steps * dt
        x = np.arange(N) * h
        X, Y = np.meshgrid(x, x, indexing="xy")

        def exact(t):
            s2 = s0 ** 2 + 2 * Dp * t
            out = 0.0
            for a in (-1, 0, 1):
                for b in (-1, 0, 1):
                    out = out + s0 ** 2 / s2 * np.exp(-((X - x0[0] - vp[0] * t - a) ** 2 +
                                                        (Y - x0[1] - vp[1] * t - b) ** 2) / (2 * s2))
            return out

        lat = _lattice(orc, N, tau, v=(vp[0] * dt / h, vp[1] * dt / h))
        fs = lat.init(exact(0.0))
        for _ in range(steps):
            fs, _ = lat.substep(fs)
        errs.append(np.abs(lat.concentration(fs) - exact(T)).max())
    orders = np.log2(np.asarray(errs[:-1]) / np.asarray(errs[1:]))
    assert np.all((orders > 1.8) & (orders < 2.2)), orders


@pytest.mark.parametrize("D,t1,t2", [(1e-2, 400, 600), (5e-3, 700, 900), (0.1, 60, 120)])
def test_relaxation_time_gives_the_diffusion_coefficient(orc, D, t1, t2):
    """Sec. 4.1 relates the relaxation time to the diffusion coefficient.
    The oracle's own mapping tau(D) is checked against what the scheme does:
    on a periodic box at rest, once the non-equilibrium start has decayed,
    the spatial variance of a pulse grows by exactly 2 D per fine step (the
    discrete second-moment balance).  A wrong mapping, e.g. D/c_s^2 with
    c_s^2 = 1 or 1/2, is off by a factor of 3 or 1.5."""
    tau = orc.relaxation_time(D)
    N = 96
    x = np.arange(N, dtype=np.float64)
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = np.exp(-((X - 47.5) ** 2 + (Y - 47.5) ** 2) / (2 * 4.0 ** 2))
    lat = _lattice(orc, N, tau)
    fs = lat.init(u0)

    def var_x(fs):
        u = lat.concentration(fs)
        m = u.sum()
        cx = (u * X).sum() / m
        return (u * (X - cx) ** 2).sum() / m

    v = {}
    for n in range(1, t2 + 1):
        fs, _ = lat.substep(fs)
        if n in (t1, t2):
            v[n] = var_x(fs)
    D_meas = (v[t2] - v[t1]) / (2.0 * (t2 - t1))
    assert abs(D_meas / D - 1.0) < 1e-6, (D_meas, D, tau)
    assert abs(orc.sound_speed_sq() - 1.0 / 3.0) < 1e-15


@pytest.mark.parametrize("sx,sy", [(-1, 0), (1, 0), (0, -1), (0, 1), (-1, -1), (1, -1), (-1, 1), (1, 1)])
def test_maxent_neumann_normal_matches_edge_form(orc, sx, sy):
    """The closure for a real unit normal reproduces the patch-edge form
    (integer direction) bit for bit at axis and diagonal normals."""
    ex, ey, _, _ = orc.d2q9()
    rng = np.random.default_rng(40 + 3 * sx + sy)
    unknown = sum(1 << q for q in range(9) if ex[q] * sx + ey[q] * sy < 0 or (sx and sy and ex[q] * sx + ey[q] * sy == 0
                                                                              and q > 0))
    f = rng.uniform(0.05, 0.3, 9)
    fs = rng.uniform(0.05, 0.3, 9)
    n = np.hypot(sx, sy)
    a, ia = orc.maxent_neumann(f, unknown, sx, sy, -0.02, fs)
    b, ib = orc.maxent_neumann_normal(f, unknown, sx / n, sy / n, -0.02, fs)
    assert ia == ib == 0 and np.array_equal(a, b)


@pytest.mark.parametrize("theta", [0.3, 1.1, 2.0, 3.9, 5.5])
def test_maxent_neumann_curved_normal(orc, theta):
    """eq. (LBM_Neu) at a curved impermeable wall (q^p = 0, normal at an
    angle the lattice does not resolve): the unknowns with e.n < 0 are the
    minimiser of H under the flux constraint (generic optimiser), KKT holds
    with one gamma, the normal flux of the closed node is zero, and the
    unknown links with e.n >= 0 (grazed by the wall) are bounced back."""
    from scipy.optimize import minimize
    ex, ey, w, opp = orc.d2q9()
    nx, ny = np.cos(theta), np.sin(theta)
    a = ex * nx + ey * ny
    rng = np.random.default_rng(int(theta * 100))
    # populations that stream out of the wall: e.n < 0, plus the link with
    # the smallest positive e.n (a grazing link whose upstream node is solid)
    Mm = [q for q in range(1, 9) if a[q] < 0]
    graze = min((q for q in range(1, 9) if a[q] >= 0), key=lambda q: a[q])
    unknown = sum(1 << q for q in Mm) | (1 << graze)
    f = rng.uniform(0.05, 0.3, 9)
    fs = rng.uniform(0.05, 0.3, 9)
    out, inf = orc.maxent_neumann_normal(f, unknown, nx, ny, 0.0, fs)
    assert inf == 0
    assert out[graze] == fs[opp[graze]]
    assert abs(np.dot(out, a)) <= 1e-13 * np.sum(np.abs(a * out))
    gam = -(np.log(out[Mm] / w[Mm]) + 1.0) / a[Mm]
    assert np.ptp(gam) < 1e-11 * max(1.0, abs(gam[0]))
    assert np.all(out[Mm] > 0)
    rhs = -sum(a[q] * out[q] for q in range(9) if q not in Mm)
    res = minimize(lambda z: _h(z, w[Mm]), x0=np.full(len(Mm), 0.1),
                   constraints=[{"type": "eq", "fun": lambda z: np.dot(z, a[Mm]) - rhs}],
                   bounds=[(1e-14, None)] * len(Mm), method="SLSQP", options={"ftol": 1e-15, "maxiter": 500})
    assert np.allclose(res.x, out[Mm], rtol=1e-5)


def test_wall_closure_zero_flux_on_the_lattice(orc):
    """On a pore lattice (disks, flow, near-equilibrium state), after
    streaming, the wall closure leaves every interior fluid node next to a
    grain with zero normal flux sum_q (e_q.n) f_q and positive populations
    in M- (all e_q.n < 0, where the other populations carry flux into the
    wall), keeps bounce-back on the links the wall grazes, and changes the
    bounce-back values elsewhere."""
    from paper_1601_02708_amd import inputs
    ex, ey, w, _ = orc.d2q9()
    N = 65
    pack = inputs.random_disks(N, 0.75, seed=3, r_min=3, r_max=7)
    wn = inputs.wall_normals(pack)
    rng = np.random.default_rng(5)
    vx = rng.uniform(-0.04, 0.04, (N, N))
    vy = rng.uniform(-0.04, 0.04, (N, N))
    lat = orc.Lattice(N, 0.7, vx, vy, solid=pack.solid, wall_normals=wn)
    u = rng.uniform(0.5, 1.5, (N, N))
    fs = w[:, None, None] * u[None] * (1 + 0.05 * rng.standard_normal((9, N, N)))
    fs[:, pack.solid != 0] = 0.0
    f, _ = lat.stream(fs)
    bb = f.copy()
    inf = orc.lib().orc_apply_wall_closure(lat.ptr, fs.ctypes.data, f.ctypes.data)
    solid = pack.solid != 0
    checked = 0
    for j in range(1, N - 1):
        for i in range(1, N - 1):
            if solid[j, i]:
                continue
            S = [q for q in range(1, 9) if solid[j - ey[q], i - ex[q]]]
            if not S:
                continue
            a = ex * wn[0, j, i] + ey * wn[1, j, i]
            Mm = [q for q in range(1, 9) if a[q] < 0]            # the unknowns of eq. (LBM_Neu)
            for q in S:
                if a[q] >= 0:                                      # grazed link: bounce-back
                    assert f[q, j, i] == bb[q, j, i]
            known_flux = sum(a[q] * f[q, j, i] for q in range(9) if q not in Mm)
            if known_flux <= 0:
                continue
            assert abs(np.dot(a, f[:, j, i])) <= 1e-13 * np.sum(np.abs(a * f[:, j, i]))
            assert all(f[q, j, i] > 0 for q in Mm)
            checked += 1
    assert checked > 200 and inf >= 0
    assert not np.array_equal(f, bb)
