"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it pins.  None of them re-types an oracle
formula: they use worked values printed in the paper, exact identities,
brute-force alternatives, closed forms derived independently, and
convergence behaviour the paper states.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import interp, lattice, mesh, physics, solver, tgv, treeid

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


# ---------------------------------------------------------------- P1 -------
def test_partition_figure_worked_example():
    """Sec. 3.1, domain-decomposition figure: Z order, weights, cumulative
    weights and the three-process split printed in the figure."""
    import json
    with open(f"{GOLDEN}/partition_figure.json") as fh:
        g = json.load(fh)
    spec = W.partition_example()
    ids, w, W_, proc = treeid.partition(spec.leaf_ids, 2, g["nproc"])
    assert [int(v) for v in ids] == g["sorted_tree_ids"]
    assert list(w) == g["weights"]
    assert list(W_) == g["cumulative_weights"]
    groups = [[int(t) for t, p in zip(ids, proc) if p == k]
              for k in range(1, g["nproc"] + 1)]
    assert groups == g["distribution"]


def test_treeid_decode_matches_recursive_enumeration():
    """Brute force: enumerate the tree recursively (children of t are
    2^d t + 1 .. 2^d t + 2^d, child k at offset bits of k) and compare."""
    for d in (2, 3):
        ids, pos = [0], [(0, (0,) * d)]
        frontier = [(0, 0, (0,) * d)]
        for _ in range(3 if d == 3 else 4):
            nxt = []
            for t, L, c in frontier:
                for k in range(1 << d):
                    child = (1 << d) * t + 1 + k
                    cc = tuple(2 * c[a] + ((k >> a) & 1) for a in range(d))
                    ids.append(child)
                    pos.append((L + 1, cc))
                    nxt.append((child, L + 1, cc))
            frontier = nxt
        levels, coords = treeid.decode(np.array(ids, dtype=np.uint64), d)
        for i, (L, c) in enumerate(pos):
            assert levels[i] == L and tuple(coords[i]) == c


# ---------------------------------------------------------------- P2/P3 ----
@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
def test_lattice_isotropy(name):
    lat = lattice.get(name)
    c, w = lat.c.astype(float), lat.w
    d = lat.d
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(d) / 3, atol=1e-15)
    m4 = np.einsum("i,ia,ib,ig,id->abgd", w, c, c, c, c)
    eye = np.eye(d)
    iso = (np.einsum("ab,gd->abgd", eye, eye) + np.einsum("ag,bd->abgd", eye, eye)
           + np.einsum("ad,bg->abgd", eye, eye)) / 9
    assert np.allclose(m4, iso, atol=1e-15)
    for i in range(lat.q):
        assert (lat.c[lat.opp[i]] == -lat.c[i]).all()


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
def test_equilibrium_moments(name):
    """Eq. feq with the '-u.u' reading: sum f^eq = rho, sum c f^eq = rho u,
    sum cc f^eq = rho cs2 I + rho u u exactly (the printed '+' sign fails the
    first identity)."""
    lat = lattice.get(name)
    g = torch.Generator().manual_seed(3)
    n = 64
    rho = 1 + 0.1 * torch.rand(n, generator=g, dtype=torch.float64)
    u = 0.1 * (torch.rand(lat.d, n, generator=g, dtype=torch.float64) - 0.5)
    feq = physics.equilibrium(rho, u, lat)
    r2, u2 = physics.moments(feq, lat)
    assert torch.allclose(r2, rho, rtol=0, atol=1e-15)
    assert torch.allclose(u2, u, rtol=0, atol=1e-15)
    P = physics.second_moment(feq, lat)
    expect = rho[None, None] * (torch.eye(lat.d, dtype=torch.float64)[:, :, None] / 3
                                + u[:, None] * u[None, :])
    assert torch.allclose(P, expect, atol=1e-15)
    # the printed sign gives a density off by rho u.u / cs2 * sum w /... != rho
    cu = lat.c_t() @ u
    uu = (u * u).sum(0)
    wrong = lat.w_t()[:, None] * rho * (1 + 3 * cu + 4.5 * cu * cu + 1.5 * uu)
    assert (wrong.sum(0) - rho).abs().max() > 1e-4


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
def test_strain_of_chapman_enskog_fneq_is_identity(name):
    """Sec. 2.1 strain formula applied to the Chapman-Enskog f^neq(S)
    returns S for any symmetric S and any omega."""
    lat = lattice.get(name)
    g = torch.Generator().manual_seed(5)
    n = 32
    A = torch.randn(lat.d, lat.d, n, generator=g, dtype=torch.float64) * 1e-3
    S = 0.5 * (A + A.transpose(0, 1))
    rho = 1 + 0.05 * torch.rand(n, generator=g, dtype=torch.float64)
    u = 0.05 * torch.randn(lat.d, n, generator=g, dtype=torch.float64)
    for omega in (0.7, 1.0, 1.9):
        f = physics.equilibrium(rho, u, lat) + physics.fneq_from_strain(rho, S, omega, lat)
        r2, u2, S2, _ = physics.strain_rate(f, omega, lat)
        assert (S2 - S).abs().max() < 1e-14  # roundoff of f - f^eq with f ~ 1/3
        assert torch.allclose(r2, rho, atol=1e-15)
        assert torch.allclose(u2, u, atol=1e-15)


# ---------------------------------------------------------------- P4 -------
def _quad_field(d, seed):
    """Random quadratic velocity u(x) = a + B x + quadratic terms; returns
    callables u(x) -> (n, d) and S(x) = sym grad u -> (n, d, d)."""
    rng = np.random.default_rng(seed)
    a = rng.normal(size=d) * 0.02
    B = rng.normal(size=(d, d)) * 0.01
    C = rng.normal(size=(d, d, d)) * 0.003
    C = 0.5 * (C + C.transpose(0, 2, 1))       # u_m = ... + C[m,a,b] x_a x_b

    def u(x):
        x = np.atleast_2d(x)
        return a + x @ B.T + np.einsum("mab,na,nb->nm", C, x, x)

    def S(x):
        x = np.atleast_2d(x)
        grad = B[None] + 2 * np.einsum("mab,nb->nma", C, x)   # d u_m / d x_a
        return 0.5 * (grad + grad.transpose(0, 2, 1))

    return u, S


def _pdf(lat, rho, u, S, omega):
    rho_t = torch.full((len(u),), rho, dtype=torch.float64)
    u_t = torch.tensor(u, dtype=torch.float64).t()
    S_t = torch.tensor(S, dtype=torch.float64).permute(1, 2, 0)
    return (physics.equilibrium(rho_t, u_t, lat)
            + physics.fneq_from_strain(rho_t, S_t, omega, lat))


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("kind", ["gfc", "gff"])
def test_compact_interpolation_exact_on_quadratic_fields(name, kind):
    """Eqs. compact_3D_u / compact_3D_s and Steps 1-5: with constant rho and
    a quadratic velocity field (linear strain rate), the ghost pdfs equal
    f^eq(rho, u(x_t)) + f^neq(rho, S(x_t) dt_t/dt_s) at the target level's
    omega, for every octant."""
    lat = lattice.get(name)
    d = lat.d
    rho = 1.013
    omega_c, omega_f = 1 / 0.56, 1 / 0.62
    for seed in range(3):
        u, S = _quad_field(d, seed)
        signs = list(np.ndindex(*(2,) * d)) if kind == "gfc" else [(1,) * d]
        for sb in signs:
            s = [2 * v - 1 for v in sb] if kind == "gfc" else [1] * d
            if d == 3:
                pos = [(0, 0, 0), (s[0], s[1], 0), (s[0], 0, s[2]), (0, s[1], s[2])]
            else:
                pos = [(0, 0), (s[0], 0), (0, s[1]), (s[0], s[1])]
            if kind == "gfc":
                target = tuple(0.25 * v for v in s)
                om_s, om_t, ratio = omega_c, omega_f, 0.5
            else:
                target = (0.5,) * d
                om_s, om_t, ratio = omega_f, omega_c, 2.0
            x0 = np.random.default_rng(seed + 10).normal(size=d) * 2
            P = np.array(pos, dtype=float) + x0
            f_src = torch.stack([_pdf(lat, rho, u(P[k]), S(P[k]), om_s)
                                 for k in range(4)], 0)
            got = interp.fill(f_src, pos, target, om_s, om_t, ratio, lat)
            xt = np.array(target) + x0
            expect = _pdf(lat, rho, u(xt), S(xt) * ratio, om_t)
            assert torch.allclose(got, expect, rtol=0, atol=2e-15), (name, kind, s)


# ---------------------------------------------------------------- P5 -------
def _closed_form_3d(uk, Sk, s):
    """Closed form derived by hand from Eqs. compact_3D_s / compact_3D_u for
    the target at s/4 (GhostFromCoarser) in the mirrored frame."""
    H, K, M, N = range(4)
    sx, sy, sz = s

    def Dx(v): return sx * (-v[H] + v[K] + v[M] - v[N]) / 2
    def Dy(v): return sy * (-v[H] + v[K] - v[M] + v[N]) / 2
    def Dz(v): return sz * (-v[H] - v[K] + v[M] + v[N]) / 2
    Sxx, Syy, Szz = Sk[:, 0, 0], Sk[:, 1, 1], Sk[:, 2, 2]
    Sxy, Syz, Sxz = Sk[:, 0, 1], Sk[:, 1, 2], Sk[:, 0, 2]
    axx, axy, axz = Dx(Sxx) / 2, Dy(Sxx), Dz(Sxx)
    bxy, byy, byz = Dx(Syy), Dy(Syy) / 2, Dz(Syy)
    cxz, cyz, czz = Dx(Szz), Dy(Szz), Dz(Szz) / 2
    bxx, ayy = Dx(Sxy) - axy / 2, Dy(Sxy) - bxy / 2
    cyy, bzz = Dy(Syz) - byz / 2, Dz(Syz) - cyz / 2
    cxx, azz = Dx(Sxz) - axz / 2, Dz(Sxz) - cxz / 2
    T = Dz(Sxy) + Dx(Syz) + Dy(Sxz)
    ayz, bxz, cxy = T - 2 * Dx(Syz), T - 2 * Dy(Sxz), T - 2 * Dz(Sxy)
    lin = (5 * uk[H] + uk[K] + uk[M] + uk[N]) / 8
    out = []
    for m, (xx, yy, zz, xy, yz, xz) in enumerate([(axx, ayy, azz, axy, ayz, axz),
                                                  (bxx, byy, bzz, bxy, byz, bxz),
                                                  (cxx, cyy, czz, cxy, cyz, cxz)]):
        out.append(lin[m] - 3 / 16 * (xx + yy + zz)
                   - 1 / 16 * (sx * sy * xy + sy * sz * yz + sx * sz * xz))
    return np.array(out)


def test_3d_solve_matches_hand_closed_form_on_random_data():
    """The assembled 30x30 system (LAPACK) agrees with an independently
    derived closed form for arbitrary (non-quadratic) source data, all
    octants -- a transposed row or wrong sign in the assembly fails here."""
    rng = np.random.default_rng(7)
    for sb in np.ndindex(2, 2, 2):
        s = [2 * v - 1 for v in sb]
        pos = [(0, 0, 0), (s[0], s[1], 0), (s[0], 0, s[2]), (0, s[1], s[2])]
        uk = rng.normal(size=(4, 3))
        A = rng.normal(size=(4, 3, 3))
        Sk = 0.5 * (A + A.transpose(0, 2, 1))
        got = interp.compact3d(pos, tuple(0.25 * v for v in s),
                               torch.tensor(uk)[None], torch.tensor(Sk)[None])[0].numpy()
        assert np.allclose(got, _closed_form_3d(uk, Sk, s), atol=1e-13)
    # GhostFromFiner: target at the centroid, s = +1
    pos = [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
    uk = rng.normal(size=(4, 3))
    A = rng.normal(size=(4, 3, 3))
    Sk = 0.5 * (A + A.transpose(0, 2, 1))
    got = interp.compact3d(pos, (0.5, 0.5, 0.5), torch.tensor(uk)[None],
                           torch.tensor(Sk)[None])[0].numpy()
    axx = (-Sk[0, 0, 0] + Sk[1, 0, 0] + Sk[2, 0, 0] - Sk[3, 0, 0]) / 4
    byy = (-Sk[0, 1, 1] + Sk[1, 1, 1] - Sk[2, 1, 1] + Sk[3, 1, 1]) / 4
    czz = (-Sk[0, 2, 2] - Sk[1, 2, 2] + Sk[2, 2, 2] + Sk[3, 2, 2]) / 4
    # GhostFromFiner closed form needs all nine diagonal coefficients
    Dx = lambda v: (-v[0] + v[1] + v[2] - v[3]) / 2
    Dy = lambda v: (-v[0] + v[1] - v[2] + v[3]) / 2
    Dz = lambda v: (-v[0] - v[1] + v[2] + v[3]) / 2
    S_ = lambda a, b: Sk[:, a, b]
    ayy = Dy(S_(0, 1)) - Dx(S_(1, 1)) / 2
    azz = Dz(S_(0, 2)) - Dx(S_(2, 2)) / 2
    bxx = Dx(S_(0, 1)) - Dy(S_(0, 0)) / 2
    bzz = Dz(S_(1, 2)) - Dy(S_(2, 2)) / 2
    cxx = Dx(S_(0, 2)) - Dz(S_(0, 0)) / 2
    cyy = Dy(S_(1, 2)) - Dz(S_(1, 1)) / 2
    expect = uk.mean(0) - 0.25 * np.array([axx + ayy + azz, bxx + byy + bzz,
                                           cxx + cyy + czz])
    assert np.allclose(got, expect, atol=1e-13)


def test_2d_interpolation_closed_forms():
    """2D reading: GhostFromCoarser u = (9,3,3,1)/16 corners - 3/16 (a_xx +
    a_yy); GhostFromFiner u = mean - 1/4 (a_xx + a_yy), with square-averaged
    strain differences."""
    rng = np.random.default_rng(11)
    for sb in np.ndindex(2, 2):
        s = [2 * v - 1 for v in sb]
        pos = [(0, 0), (s[0], 0), (0, s[1]), (s[0], s[1])]
        uk = rng.normal(size=(4, 2))
        A = rng.normal(size=(4, 2, 2))
        Sk = 0.5 * (A + A.transpose(0, 2, 1))
        Dx = lambda v: s[0] * (-v[0] + v[1] - v[2] + v[3]) / 2
        Dy = lambda v: s[1] * (-v[0] - v[1] + v[2] + v[3]) / 2
        axx, axy = Dx(Sk[:, 0, 0]) / 2, Dy(Sk[:, 0, 0])
        bxy, byy = Dx(Sk[:, 1, 1]), Dy(Sk[:, 1, 1]) / 2
        bxx, ayy = Dx(Sk[:, 0, 1]) - axy / 2, Dy(Sk[:, 0, 1]) - bxy / 2
        lin = (9 * uk[0] + 3 * uk[1] + 3 * uk[2] + uk[3]) / 16
        expect = lin - 3 / 16 * np.array([axx + ayy, bxx + byy])
        got = interp.compact2d(pos, (0.25 * s[0], 0.25 * s[1]),
                               torch.tensor(uk)[None], torch.tensor(Sk)[None])[0].numpy()
        assert np.allclose(got, expect, atol=1e-13)
    pos = [(0, 0), (1, 0), (0, 1), (1, 1)]
    got = interp.compact2d(pos, (0.5, 0.5), torch.tensor(uk)[None],
                           torch.tensor(Sk)[None])[0].numpy()
    Dx = lambda v: (-v[0] + v[1] - v[2] + v[3]) / 2
    Dy = lambda v: (-v[0] - v[1] + v[2] + v[3]) / 2
    axx, axy = Dx(Sk[:, 0, 0]) / 2, Dy(Sk[:, 0, 0])
    bxy, byy = Dx(Sk[:, 1, 1]), Dy(Sk[:, 1, 1]) / 2
    bxx, ayy = Dx(Sk[:, 0, 1]) - axy / 2, Dy(Sk[:, 0, 1]) - bxy / 2
    expect = uk.mean(0) - 0.25 * np.array([axx + ayy, bxx + byy])
    assert np.allclose(got, expect, atol=1e-13)


# ------------------------------------------------------ mesh-level fills ----
def _level_fields(m, L, u_fn, S_fn, rho):
    t = m.lev(L)
    pos = m.positions(L)
    scale = 2.0 ** -(L - m.level0)
    return pos, u_fn(pos), S_fn(pos) * scale


@pytest.mark.parametrize("spec_fn", [
    lambda: W.refined_box_mesh("D2Q9", 5, 8, 24),
    lambda: W.refined_box_mesh("D3Q19", 4, 4, 12),
    lambda: W.refined_box_mesh("D3Q27", 4, 4, 12),
])
def test_mesh_fill_exact_on_quadratic_field(spec_fn):
    """The sync fill of a whole mesh (source tables, octant signs, target
    positions, rescaling) reproduces a quadratic field at every ghost."""
    m = mesh.build(spec_fn())
    d = m.d
    u_fn, S_fn = _quad_field(d, 42)
    # keep the field small so pdfs stay positive; positions in coarse units
    sim = solver.OracleSim(m, 0.57)
    rho = 0.98
    for L in range(m.level0, m.lmax + 1):
        pos, uu, SS = _level_fields(m, L, lambda p: u_fn(p / 16.0) * 0.5,
                                    lambda p: S_fn(p / 16.0) * 0.5 / 16.0, rho)
        sim.f[L] = _pdf(m.lattice, rho, uu, SS, sim.omega[L])
        t = m.lev(L)
        sim.f[L][:, t.n_fluid:] = float("nan")
        sim.f[L] = sim.f[L].clone()
    expect = {}
    for L in range(m.level0, m.lmax + 1):
        pos, uu, SS = _level_fields(m, L, lambda p: u_fn(p / 16.0) * 0.5,
                                    lambda p: S_fn(p / 16.0) * 0.5 / 16.0, rho)
        expect[L] = _pdf(m.lattice, rho, uu, SS, sim.omega[L])
    sim.fill_all()
    for L in range(m.level0, m.lmax + 1):
        t = m.lev(L)
        got = sim.f[L][:, t.n_fluid:]
        assert not torch.isnan(got).any()
        assert torch.allclose(got, expect[L][:, t.n_fluid:], rtol=0, atol=1e-14)


# ------------------------------------------------------ neighbour tables ----
def test_neighbour_table_brute_force():
    """Brute force over all element pairs: nbr[i][x] is the element at
    x - c_i (periodic), on a small two-level 2D mesh and a 3D mesh."""
    for spec in (W.refined_box_mesh("D2Q9", 3, 2, 6),
                 W.refined_box_mesh("D3Q19", 3, 2, 6)):
        m = mesh.build(spec)
        for t in m.levels:
            n_side = spec.box_extent[0] << (t.level - m.level0)
            pos = {tuple(c): k for k, c in enumerate(t.coords)}
            for x in range(t.n):
                for i in range(m.lattice.q):
                    y = tuple((t.coords[x] - m.lattice.c[i]) % n_side)
                    want = pos.get(y, mesh.MISSING)
                    assert t.nbr[i, x] == want


def test_sphere_mesh_codes():
    """Sphere channel: bounce-back next to solid cells, equilibrium on the
    inflow/lateral faces, copy on the outlet; no active element misses a
    neighbour."""
    spec = W.sphere_channel_mesh(8, 2, l0_per_d=4, length=(-2.0, 3.0),
                                 half_width=2.0, boxes_in_d=((-1.0, 1.5, 1.0),))
    m = mesh.build(spec)
    fine = m.lev(m.lmax)
    assert (fine.nbr == mesh.BOUNCE).sum() > 0
    coarse = m.lev(m.level0)
    assert (coarse.nbr == mesh.EQ).any() and (coarse.nbr == mesh.COPY).any()
    # every bounce link points at a solid cell
    for i in range(m.lattice.q):
        xs = np.where(fine.nbr[i] == mesh.BOUNCE)[0]
        for x in xs[:50]:
            c = fine.coords[x] - m.lattice.c[i]
            key = c[0] + (c[1] << m.lmax) + (c[2] << (2 * m.lmax))
            assert key in set(fine.solid_keys.tolist())


# ------------------------------------------------------------ physics -------
def _tgv_sim(spec, n0, u0, tau0, poison=True):
    m = mesh.build(spec)
    sim = solver.OracleSim(m, tau0, poison=poison)
    rho, u, S = {}, {}, {}
    for L in range(m.level0, m.lmax + 1):
        t = m.lev(L)
        pos = m.positions(L)[:t.n_fluid]
        r, uu, SS = W.tgv_fields(pos, n0, u0)
        rho[L], u[L], S[L] = r, uu, SS * 2.0 ** -(L - m.level0)
    sim.init(rho, u, S)
    return sim


def test_single_level_matches_roll_streaming():
    """Limit case: a one-level periodic mesh is plain periodic BGK; compare
    with streaming by array shifts on the Cartesian grid."""
    for spec, n in ((W.uniform_box_mesh("D2Q9", 4), 16),
                    (W.uniform_box_mesh("D3Q19", 3), 8)):
        sim = _tgv_sim(spec, n, 0.05, 0.7)
        m = sim.mesh
        lat = m.lattice
        t = m.lev(m.level0)
        grid_idx = np.zeros((n,) * lat.d, dtype=np.int64)
        for k, c in enumerate(t.coords):
            grid_idx[tuple(c)] = k
        f = sim.f[m.level0].numpy()[:, grid_idx]      # (q, n, n[, n])
        omega = sim.omega[m.level0]
        for _ in range(5):
            rho = f.sum(0)
            u = np.einsum("ia,i...->a...", lat.c, f) / rho
            cu = np.einsum("ia,a...->i...", lat.c, u)
            uu = (u * u).sum(0)
            w = lat.w.reshape((-1,) + (1,) * lat.d)
            feq = w * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
            fs = f - omega * (f - feq)
            f = np.stack([np.roll(fs[i], tuple(lat.c[i]), axis=tuple(range(lat.d)))
                          for i in range(lat.q)])
            sim.step(1)
        got = sim.f[m.level0].numpy()[:, grid_idx]
        assert np.allclose(got, f, rtol=0, atol=1e-15)


def test_mass_conserved_single_level():
    """Single-level periodic BGK conserves mass to roundoff (1000 steps)."""
    sim = _tgv_sim(W.uniform_box_mesh("D2Q9", 5), 32, 0.02, 0.8)
    M0 = float(sim.mass())
    sim.step(1000)
    assert abs(float(sim.mass()) - M0) / M0 < 1e-12


def test_uniform_flow_preserved_multilevel():
    """A uniform flow (f^neq = 0) is a fixed point of the multilevel step:
    the fills reproduce constants."""
    for spec in (W.refined_box_mesh("D2Q9", 4, 4, 12),
                 W.refined_box_mesh("D3Q19", 3, 2, 6)):
        m = mesh.build(spec)
        d = m.d
        uc = np.array([0.03, -0.02, 0.01][:d])
        sim = solver.OracleSim(m, 0.6)
        rho, u, S = {}, {}, {}
        for L in range(m.level0, m.lmax + 1):
            nf = m.lev(L).n_fluid
            rho[L], u[L], S[L] = W.uniform_fields(nf, d, uc)
        sim.init(rho, u, S)
        sim.step(4)
        lat = m.lattice
        feq = physics.equilibrium(torch.ones(1, dtype=torch.float64),
                                  torch.tensor(uc)[:, None], lat)
        for L in range(m.level0, m.lmax + 1):
            assert torch.allclose(sim.f[L], feq.expand_as(sim.f[L]), atol=1e-15)


@pytest.mark.parametrize("spec_fn,n0,steps", [
    (lambda: W.refined_box_mesh("D2Q9", 5, 8, 24), 32, 200),
    (lambda: W.refined_box_mesh("D3Q19", 4, 4, 12), 16, 12),
    (lambda: W.refined_box_mesh("D2Q9", 5, 8, 24, extra_levels=[(20, 44)]), 32, 12),
    (lambda: W.refined_box_mesh("D3Q19", 4, 2, 14, extra_levels=[(10, 18)]), 16, 3),
    (lambda: W.refined_box_mesh("D3Q27", 4, 2, 14, extra_levels=[(10, 18)]), 16, 3),
])
def test_nan_poisoning_never_reaches_fluid(spec_fn, n0, steps):
    """Ghost slots start as NaN and missing pull sources give NaN; after full
    runs of the recursive schedule no fluid pdf is NaN (every value a fluid
    element reads was filled at the right time)."""
    sim = _tgv_sim(spec_fn(), n0, 0.02, 0.7)
    for _ in range(steps):
        sim.step(1)
        for L in range(sim.L0, sim.Lmax + 1):
            nf = sim.mesh.lev(L).n_fluid
            assert not torch.isnan(sim.f[L][:, :nf]).any()


def test_single_level_tgv_decays_at_bgk_viscosity():
    """Sec. 4.1 / Eq. nu: a single-level TGV decays with nu = (tau-1/2)/3;
    the error at t_D is second order (diffusive scaling, tau fixed)."""
    errs = []
    for lev in (4, 5):
        n0 = 1 << lev
        u0 = 0.02 * 8 / n0
        sim = _tgv_sim(W.uniform_box_mesh("D2Q9", lev), n0, u0, 0.8)
        nu0 = tgv.nu_from_tau(0.8)
        sim.step(int(round(tgv.decay_time(n0, nu0))))
        errs.append(tgv.errors(sim, n0, u0, nu0)[0])
    assert errs[1] < 2e-3
    assert 3.5 < errs[0] / errs[1] < 4.5


@pytest.mark.slow
def test_tgv_second_order_convergence_half_refined():
    """Sec. 4.1 convergence study (left half level L, right half L+1):
    velocity and strain rate converge at second order."""
    eu, es = [], []
    for lev in (4, 5, 6):
        n0 = 1 << lev
        u0 = 0.02 * 8 / n0
        sim = _tgv_sim(W.half_refined_2d(lev), n0, u0, 0.8)
        nu0 = tgv.nu_from_tau(0.8)
        sim.step(int(round(tgv.decay_time(n0, nu0))))
        a, b = tgv.errors(sim, n0, u0, nu0)
        eu.append(a)
        es.append(b)
    su = [math.log2(eu[i] / eu[i + 1]) for i in range(2)]
    ss = [math.log2(es[i] / es[i + 1]) for i in range(2)]
    assert all(1.8 < s < 2.4 for s in su), su
    assert all(1.8 < s < 2.4 for s in ss), ss


def test_mass_drift_multilevel_is_small():
    """Multilevel mass is not exactly conserved by the interpolation scheme
    (the exactly conservative schemes are the volumetric ones, Sec. 1); the
    drift on the D2Q9 refined TGV stays at the 1e-6 level."""
    sim = _tgv_sim(W.refined_box_mesh("D2Q9", 5, 8, 24), 32, 0.01, 0.8)
    M0 = float(sim.mass())
    sim.step(100)
    drift = abs(float(sim.mass()) - M0) / M0
    assert drift < 1e-5


# ------------------------------------------ curved walls (Sec. 2.3) --------
def _channel_wall_offset(stencil, q_low, q_high, h=24, tau=0.8):
    """Effective distance between the walls, from the decay rate of the
    lowest shear mode, minus the distance the wall fractions place them at."""
    spec = W.plane_channel_mesh(stencil, 5, 2, h)
    m = mesh.build(spec)
    walls = W.plane_wall_links(spec, m.lattice.c, q_low, q_high)
    z_lo = 1.5 - q_low
    H = (h - 1.5 + q_high) - z_lo
    sim = solver.OracleSim(m, tau, walls=walls)
    pos = m.positions(5)[:m.lev(5).n_fluid]
    r, u, S = W.shear_wave_fields(pos, z_lo, H, 0.01)
    sim.init({5: r}, {5: u}, {5: S})
    sim.step(400)
    e1 = float(sim.kinetic_energy())
    sim.step(1200)
    e2 = float(sim.kinetic_energy())
    nu = (tau - 0.5) / 3.0
    rate = math.log(e1 / e2) / (2 * 1200)          # energy decays at 2 nu k^2
    return math.pi * math.sqrt(nu / rate) - H


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("q_low,q_high", [(0.25, 0.25), (0.75, 0.75), (0.1, 0.9)])
def test_curved_wall_sits_where_the_fraction_puts_it(stencil, q_low, q_high):
    """Sec. 2.3 (linear interpolated bounce-back): a shear wave between two
    parallel walls decays as exp(-nu (pi/H)^2 t) with H the distance between
    the walls.  The walls are placed by the fractions alone (the solid rows
    do not move), so the measured H must follow q to well under the quarter
    cell that separates the cases; halfway bounce-back would give H = 22
    for all of them.  Measured offset: about -0.012 cells at h = 24."""
    off = _channel_wall_offset(stencil, q_low, q_high)
    assert abs(off) < 0.05, off


def _compact_sphere(stencil="D3Q19"):
    return W.sphere_channel_mesh(8, 2, l0_per_d=4, length=(-1.5, 2.0), half_width=1.5,
                                 boxes_in_d=((-0.75, 1.0, 0.75),), stencil=stencil)


def test_wall_fraction_one_half_is_halfway_bounce_back():
    """At q = 1/2 both branches of the interpolated rule reduce to halfway
    bounce-back: runs with and without the fractions agree exactly, state
    and momentum-exchange force."""
    spec = _compact_sphere()
    m = mesh.build(spec)
    ids, dirs, q = W.sphere_wall_links(spec, m.lattice.c)
    assert len(ids) > 100
    out = []
    for walls in (None, (ids, dirs, np.full(len(q), 0.5))):
        sim = solver.OracleSim(m, 0.6, u_in=[0.04, 0.0, 0.0], walls=walls)
        rho, u, S = {}, {}, {}
        for L in range(m.level0, m.lmax + 1):
            nf = m.lev(L).n_fluid
            rho[L], u[L], S[L] = np.ones(nf), np.zeros((nf, 3)), np.zeros((nf, 3, 3))
            u[L][:, 0] = 0.04
        sim.init(rho, u, S)
        sim.step(3)
        out.append((sim.f[m.lmax].clone(), sim.force()))
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])


def test_fluid_at_rest_stays_at_rest_with_curved_walls():
    """The interpolation weights of each branch sum to one, so fluid at
    rest next to walls at any fractions stays at rest and feels no force."""
    spec = _compact_sphere()
    m = mesh.build(spec)
    ids, dirs, q = W.sphere_wall_links(spec, m.lattice.c)
    assert q.min() < 0.2 and q.max() > 0.8
    sim = solver.OracleSim(m, 0.6, walls=(ids, dirs, q))
    rho, u, S = {}, {}, {}
    for L in range(m.level0, m.lmax + 1):
        nf = m.lev(L).n_fluid
        rho[L], u[L], S[L] = np.ones(nf), np.zeros((nf, 3)), np.zeros((nf, 3, 3))
    sim.init(rho, u, S)
    sim.step(3)
    w = m.lattice.w_t(torch.float64)[:, None]
    for L in range(m.level0, m.lmax + 1):
        nf = m.lev(L).n_fluid
        assert (sim.f[L][:, :nf] - w).abs().max() < 1e-15
    assert sim.force().abs().max() < 1e-13


# ------------------------------- momentum-exchange force (Sec. 2.3) --------
def _channel_fields(pos, width, height, d):
    """A smooth, non-symmetric state of a channel: density bump, shear along
    the walls and flow towards them (every force component is non-zero)."""
    x = 2 * math.pi * pos[:, 0] / width
    z = math.pi * pos[:, d - 1] / height
    rho = 1.0 + 0.01 * np.sin(x) * np.cos(z) + 0.004 * np.cos(2 * z)
    u = np.zeros((len(pos), d))
    u[:, 0] = 0.03 * np.sin(z) + 0.01 * np.cos(x)
    u[:, d - 1] = 0.02 * np.sin(x) * np.sin(2 * z) + 0.005
    if d == 3:
        u[:, 1] = 0.01 * np.cos(x + z)
    return rho, u, np.zeros((len(pos), d, d))


def _fluid_momentum(sim):
    L = sim.L0
    nf = sim.mesh.lev(L).n_fluid
    return sim.lat.c.astype(np.float64).T @ sim.f[L][:, :nf].numpy().sum(1)


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("walls", ["halfway", "q<1/2 and q>1/2", "random q"])
def test_force_is_the_momentum_the_walls_remove(stencil, walls):
    """Sec. 2.3 momentum exchange, pinned by momentum balance.  BGK conserves
    each element's momentum and periodic streaming only moves it, so in a
    periodic channel the fluid momentum changes over one step exactly by what
    the wall links take out (c_i f*_i(x) leaving along i) and put back (the
    returning f_opp(i)(x, t+1)): P(t+1) - P(t) = -F(t).  A dropped returning
    term, a wrong factor, sign or direction, or an interpolation rule whose
    value is not the one streamed, all break the balance."""
    d = 2 if stencil == "D2Q9" else 3
    width, h = (16, 12) if d == 2 else (6, 10)
    spec = W.plane_channel_mesh(stencil, 5, width, h)
    m = mesh.build(spec)
    wl = None
    if walls != "halfway":
        ids, dirs, q = W.plane_wall_links(spec, m.lattice.c, 0.3, 0.8)
        if walls == "random q":
            q = np.random.default_rng(7).uniform(0.0, 1.0, len(q))
        wl = (ids, dirs, q)
    sim = solver.OracleSim(m, 0.7, walls=wl)
    pos = m.positions(5)[:m.lev(5).n_fluid]
    r, u, S = _channel_fields(pos, width, h, d)
    sim.init({5: r}, {5: u}, {5: S})
    for _ in range(6):
        F = sim.force().numpy()
        P0 = _fluid_momentum(sim)
        sim.step(1)
        P1 = _fluid_momentum(sim)
        assert np.abs(F).min() > 1e-6          # every component is exercised
        assert np.abs((P1 - P0) + F).max() < 1e-13, (P1 - P0, F)


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
def test_force_level_scaling_closed_form(stencil):
    """Sec. 2.3 force on a two-level channel, the lower wall on the coarse
    level and the upper wall on the fine level (the fine band spans the
    periodic directions, so no ghost touches a wall).  For an equilibrium
    state with velocity u along the walls and density rho(y), halfway
    bounce-back returns f*_i = f^eq_i, and summing 2 c_i f^eq_i over the
    directions into a wall gives, per wall cell, -rho/3 (lower) or +rho/3
    (upper) normal to the wall and rho u_x/3 along it, on every one of the
    three lattices.  Each level's sum is in its own lattice units; a force
    scales as dx^(d-1) when dx/dt is level invariant, so in finest-level
    units a coarse wall cell counts 2^(d-1) times:
        F_y = (sum_upper rho - 2^(d-1) sum_lower rho) / 3
        F_x = u_x (sum_upper rho + 2^(d-1) sum_lower rho) / 3."""
    d = 2 if stencil == "D2Q9" else 3
    w, h, L0 = (8, 8, 3) if d == 2 else (4, 8, 3)
    spec = W.two_level_channel_mesh(stencil, L0, w, h)
    m = mesh.build(spec)
    ux = 0.03
    sim = solver.OracleSim(m, 0.7)
    rho, u, S = {}, {}, {}
    wall_rho = {}
    for L in (L0, L0 + 1):
        nf = m.lev(L).n_fluid
        pos = m.positions(L)[:nf]
        rho[L] = 1.0 + 0.02 * pos[:, 1] / h + 0.01 * np.sin(2 * math.pi * pos[:, 0] / w)
        u[L] = np.zeros((nf, d))
        u[L][:, 0] = ux
        S[L] = np.zeros((nf, d, d))
        dy = 0.5 / 2 ** (L - L0)                   # half a cell of level L
        wall_rho[L] = (rho[L][pos[:, 1] < dy + 1e-9].sum(), rho[L][pos[:, 1] > h - dy - 1e-9].sum())
    sim.init(rho, u, S)
    lower = wall_rho[L0][0] * 2 ** (d - 1)
    upper = wall_rho[L0 + 1][1]
    assert wall_rho[L0][1] == 0 and wall_rho[L0 + 1][0] == 0   # one wall per level
    want = np.zeros(d)
    want[0] = ux * (upper + lower) / 3.0
    want[1] = (upper - lower) / 3.0
    got = sim.force().numpy()
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max(), (got, want)


# ------------------------------------- diffusive scaling (Sec. 2.2, end) ----
# dt_(L+1) = dt_L / 4, dx_(L+1) = dx_L / 2: four fine steps per coarse step,
# four GhostFromCoarser layers, the same tau on every level; lattice velocity
# halves and density deviation quarters per level (u dt/dx, p dt^2/dx^2).
_DIFF_MESHES = [lambda: W.refined_box_mesh("D2Q9", 5, 8, 24),
                lambda: W.refined_box_mesh("D3Q19", 4, 4, 12)]


@pytest.mark.parametrize("spec_fn", _DIFF_MESHES)
def test_diffusive_uniform_flow_and_pressure_kept(spec_fn):
    """A uniform flow at uniform pressure is a fixed point when each level
    holds it in its own lattice units; the fills must convert velocity and
    density deviation between levels for that to hold."""
    m = mesh.build(spec_fn(), gfc_layers=4)
    d = m.d
    uc = np.array([0.03, -0.02, 0.01][:d])
    drho = 0.004
    sim = solver.OracleSim(m, 0.7, scaling="diffusive")
    rho, u, S = {}, {}, {}
    for L in range(m.level0, m.lmax + 1):
        r = 2.0 ** (L - m.level0)
        rho[L], u[L], S[L] = W.uniform_fields(m.lev(L).n_fluid, d, uc / r, 1.0 + drho / (r * r))
    sim.init(rho, u, S)
    sim.step(3)
    for L in range(m.level0, m.lmax + 1):
        r = 2.0 ** (L - m.level0)
        feq = physics.equilibrium(torch.tensor([1.0 + drho / (r * r)], dtype=torch.float64),
                                  torch.tensor(uc / r)[:, None], m.lattice)
        assert torch.allclose(sim.f[L], feq.expand_as(sim.f[L]), atol=1e-15), L


@pytest.mark.parametrize("spec_fn", _DIFF_MESHES)
def test_diffusive_fill_exact_on_quadratic_field(spec_fn):
    """The sync fill under diffusive scaling reproduces a quadratic velocity
    field (linear strain) at every ghost of all four layers, each level in
    its own units: u / 2^(L-L0), S / 4^(L-L0).  At rho = 1: Step 4 rescales
    f^neq by omega and dt only, while f^neq also carries rho, whose lattice
    deviation changes between levels under this scaling (the uniform-flow
    pin covers the density conversion)."""
    m = mesh.build(spec_fn(), gfc_layers=4)
    d = m.d
    u_fn, S_fn = _quad_field(d, 42)
    sim = solver.OracleSim(m, 0.57, scaling="diffusive")
    drho = 0.0
    expect = {}
    for L in range(m.level0, m.lmax + 1):
        r = 2.0 ** (L - m.level0)
        pos = m.positions(L)
        uu = u_fn(pos / 16.0) * 0.5 / r
        SS = S_fn(pos / 16.0) * 0.5 / 16.0 / (r * r)
        expect[L] = _pdf(m.lattice, 1.0 + drho / (r * r), uu, SS, sim.omega[L])
        t = m.lev(L)
        sim.f[L] = expect[L].clone()
        sim.f[L][:, t.n_fluid:] = float("nan")
    sim.fill_all()
    for L in range(m.level0, m.lmax + 1):
        t = m.lev(L)
        got = sim.f[L][:, t.n_fluid:]
        assert not torch.isnan(got).any()
        assert torch.allclose(got, expect[L][:, t.n_fluid:], rtol=0, atol=1e-14)


@pytest.mark.parametrize("spec_fn", _DIFF_MESHES)
def test_diffusive_four_layers_feed_four_fine_steps(spec_fn):
    """NaN-poisoned run: with four layers, nothing invalid reaches a fluid
    element over four fine steps per coarse step; with two layers it does."""
    spec = spec_fn()
    d = 2 if spec.stencil == "D2Q9" else 3
    n0 = spec.box_extent[0]

    def run(layers):
        m = mesh.build(spec, gfc_layers=layers)
        sim = solver.OracleSim(m, 0.7, scaling="diffusive")
        rho, u, S = {}, {}, {}
        for L in range(m.level0, m.lmax + 1):
            r = 2.0 ** (L - m.level0)
            pos = m.positions(L)[:m.lev(L).n_fluid]
            rr, uu, SS = W.tgv_fields(pos, n0, 0.02)
            rho[L], u[L], S[L] = 1.0 + (rr - 1.0) / (r * r), uu / r, SS / (r * r)
        sim.init(rho, u, S)
        sim.step(2)
        return all(torch.isfinite(sim.f[L][:, :m.lev(L).n_fluid]).all()
                   for L in range(m.level0, m.lmax + 1))
    assert run(4)
    assert not run(2)


def test_diffusive_tgv_decays_at_the_physical_viscosity():
    """Two-level Taylor-Green vortex under diffusive scaling, each level
    initialised in its own units: the energy decays at the rate the single
    viscosity nu = (tau - 1/2)/3 (coarse units) gives, |k|^2 = 2 (2 pi/32)^2,
    to 0.2% (measured +0.014%; a fine level with the acoustic tau, or
    velocities not converted, moves it by several percent)."""
    spec = W.refined_box_mesh("D2Q9", 5, 8, 24)
    m = mesh.build(spec, gfc_layers=4)
    sim = solver.OracleSim(m, 0.8, scaling="diffusive")
    rho, u, S = {}, {}, {}
    for L in range(m.level0, m.lmax + 1):
        r = 2.0 ** (L - m.level0)
        pos = m.positions(L)[:m.lev(L).n_fluid]
        rr, uu, SS = W.tgv_fields(pos, 32, 0.01)
        rho[L], u[L], S[L] = 1.0 + (rr - 1.0) / (r * r), uu / r, SS / (r * r)
    sim.init(rho, u, S)
    sim.step(20)
    e1 = float(sim.kinetic_energy())
    sim.step(200)
    e2 = float(sim.kinetic_energy())
    rate = math.log(e1 / e2) / (2 * 200)
    want = 2 * 0.1 * (2 * math.pi / 32) ** 2
    assert abs(rate / want - 1) < 2e-3, rate / want


def test_diffusive_tgv_second_order_convergence_half_refined():
    """The mesh of the Sec. 4.1 convergence study (left half level L, right
    half L+1), run under this project's diffusive-scaling variant between
    levels (four fine steps per coarse step; Sec. 2.2 applies acoustic
    scaling and names diffusive scaling only as a possible extension), with
    u0 ~ 1/N and tau fixed and errors at t_D in coarse units: velocity and
    strain rate converge at second order."""
    eu, es = [], []
    for lev in (4, 5, 6):
        n0 = 1 << lev
        u0 = 0.02 * 8 / n0
        m = mesh.build(W.half_refined_2d(lev), gfc_layers=4)
        sim = solver.OracleSim(m, 0.8, scaling="diffusive")
        rho, u, S = {}, {}, {}
        for L in range(m.level0, m.lmax + 1):
            r = 2.0 ** (L - m.level0)
            pos = m.positions(L)[:m.lev(L).n_fluid]
            rr, uu, SS = W.tgv_fields(pos, n0, u0)
            rho[L], u[L], S[L] = 1.0 + (rr - 1.0) / (r * r), uu / r, SS / (r * r)
        sim.init(rho, u, S)
        nu0 = tgv.nu_from_tau(0.8)
        sim.step(int(round(tgv.decay_time(n0, nu0))))
        a, b = tgv.errors(sim, n0, u0, nu0)
        eu.append(a)
        es.append(b)
    su = [math.log2(eu[i] / eu[i + 1]) for i in range(2)]
    ss = [math.log2(es[i] / es[i + 1]) for i in range(2)]
    print("diffusive slopes u", su, "S", ss, "errors", eu, es)
    assert all(1.8 < s < 2.4 for s in su), su
    assert all(1.8 < s < 2.4 for s in ss), ss


def test_diffusive_mass_drift_is_small():
    """Under diffusive scaling the multilevel mass (density deviations in
    coarsest-level units) drifts at the level acoustic scaling shows:
    below 1e-5 over 100 coarse steps (measured 4.5e-6; initialising the
    fine level in coarse units instead gives 4e-5)."""
    m = mesh.build(W.refined_box_mesh("D2Q9", 5, 8, 24), gfc_layers=4)
    sim = solver.OracleSim(m, 0.8, scaling="diffusive")
    rho, u, S = {}, {}, {}
    for L in range(m.level0, m.lmax + 1):
        r = 2.0 ** (L - m.level0)
        pos = m.positions(L)[:m.lev(L).n_fluid]
        rr, uu, SS = W.tgv_fields(pos, 32, 0.02)
        rho[L], u[L], S[L] = 1.0 + (rr - 1.0) / (r * r), uu / r, SS / (r * r)
    sim.init(rho, u, S)
    m0 = float(sim.mass())
    sim.step(100)
    assert abs(float(sim.mass()) - m0) / m0 < 1e-5
