"""Parity at full size on every level, in the launch configuration the bench
times: the 20.5M-element three-level sphere channel (FP32, FP16-shift) and
the 449M-element four-level sphere channel (FP16-shift).

After one coarse step from a perturbed state, for sampled elements of every
level:

(a) the pull: the pre-collision pdfs the last stream-collide gathered equal
    the previous post-collision state taken at the neighbours found by
    coordinate among the level's treeIDs (equilibrium on the domain faces,
    halfway bounce-back from solid cells) -- bit for bit, since the pull
    only moves stored values;
(b) the collision: the stored post-collision pdfs equal Eq. bgk applied in
    FP64 by the oracle to those pre-collision pdfs, within the storage
    precision;
(c) the fills of the final synchronisation: sampled GhostFromFiner and
    GhostFromCoarser (inner and outer) ghosts equal the oracle's compact
    interpolation (Steps 1-5 of Sec. 2.2) of their four sources'
    pre-collision pdfs, collided with the ghost level's omega.

The neighbour search, the source geometry (tetrahedra from the octant
signs) and all arithmetic of the expected values are the test's and the
oracle's; the library supplies its state and its source lists.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import interp as ointerp
from oracle import lattice as olat
from oracle import physics as ophys
from oracle import treeid as otree
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _device_fields(plan, k, ext, uin, dev):
    """Perturbed free stream (level-0 wavelength of 16 cells) on the device."""
    nf = plan.info[k]["n_fluid"]
    c = torch.from_numpy(plan.export(k, "coords")[:, :nf]).to(dev, torch.float64)
    p = (c + 0.5) / float(1 << k)
    tw = 2.0 * np.pi / 16.0
    x, y, z = p[0] * tw, p[1] * tw, p[2] * tw
    rho = 1.0 + 0.002 * torch.cos(x + y)
    u = torch.empty((3, nf), dtype=torch.float64, device=dev)
    u[0] = uin + 0.01 * torch.sin(x) * torch.cos(y)
    u[1] = 0.01 * torch.cos(x) * torch.sin(z)
    u[2] = 0.005 * torch.sin(y + z)
    return rho, u


class _Level:
    """Lookup of treeIDs among a level's elements.  The layout is a sequence
    of runs each ascending by treeID ([plain fluid | source fluid | inner |
    outer | GhostFromFiner]), so each run is searched on its own."""

    def __init__(self, plan, k):
        i = plan.info[k]
        self.tid = plan.export(k, "treeid")
        nf, cb = i["n_fluid"], i["n_fluid"] - i["n_cap_fluid"]
        b = [0, cb, nf, nf + i["n_gfc_inner"], nf + i["n_gfc_inner"] + i["n_gfc_outer"], i["n"]]
        self.runs = [(b[r], b[r + 1]) for r in range(5) if b[r + 1] > b[r]]
        for lo, hi in self.runs:
            assert (np.diff(self.tid[lo:hi].astype(np.int64)) > 0).all()

    def find(self, t):
        out = np.full(len(t), -1, dtype=np.int64)
        for lo, hi in self.runs:
            run = self.tid[lo:hi]
            pos = np.minimum(np.searchsorted(run, t), len(run) - 1)
            hit = run[pos] == t
            out[hit] = lo + pos[hit]
        return out


def _take(dev_arr, rows, cols):
    """dev_arr[rows, cols] for host index arrays, on the host."""
    r = torch.as_tensor(np.ascontiguousarray(rows), device=dev_arr.device)
    c = torch.as_tensor(np.ascontiguousarray(cols), device=dev_arr.device)
    return dev_arr[r, c].cpu().numpy()


def _cols(dev_arr, cols):
    return dev_arr[:, torch.as_tensor(np.ascontiguousarray(cols), device=dev_arr.device)] \
        .cpu().numpy()


def _f16s_ok(got, expect, w, c, slack_rel=2e-6):
    """FP16-shift stores (see the stream-collide): each value within half an
    ulp (2^-11 relative) of the element's summed deviations, mass and
    momentum within the rounding of the values that absorb them."""
    g = np.abs(expect - w[:, None])
    slack = slack_rel * np.abs(expect)
    gsum = g.sum(0)
    d = got - expect
    ok = (np.abs(d) <= 2.0 ** -11 * gsum[None, :] + slack).all()
    rest = int(np.where(~c.any(1))[0][0])
    ok &= (np.abs(d.sum(0)) <= 2.0 ** -11 * g[rest] + 2.0 ** -20 * gsum + slack.sum(0)).all()
    for a in range(3):
        pa = int(np.where((c == np.eye(3, dtype=c.dtype)[a]).all(1))[0][0])
        ma = int(np.where((c == -np.eye(3, dtype=c.dtype)[a]).all(1))[0][0])
        dj = (c[:, a][:, None] * d).sum(0)
        ok &= (np.abs(dj) <= 2.0 ** -11 * (g[pa] + g[ma]) + 2.0 ** -20 * gsum
               + slack.sum(0)).all()
    return bool(ok)


def _check_levels(spec, plan, sim, precision, uin, n_sample, seed=1601):
    lat = olat.get(spec.stencil)
    c_lib, w_lib = (np.asarray(v) for v in __import__("paper_1601_06984_amd").lattice(
        spec.stencil))
    perm = np.asarray(H.direction_perm(spec.stencil, lat))   # library i -> oracle index
    to_o = np.argsort(perm)                                  # library rows in oracle order
    q, d, nl = plan.q, plan.d, plan.n_levels
    opp = np.array([int(np.where((c_lib == -c_lib[i]).all(1))[0][0]) for i in range(q)])
    ext0 = np.asarray(spec.box_extent)
    face = spec.face_bc
    rng = np.random.default_rng(seed)
    feq_in = ophys.equilibrium(torch.ones(1, dtype=torch.float64),
                               torch.tensor(np.array(uin)[:, None], dtype=torch.float64),
                               lat).numpy()[:, 0][perm]          # library order
    omega = [1.0 / ophys.level_tau(sim.tau0, plan.level0 + k, plan.level0) for k in range(nl)]
    look = [_Level(plan, k) for k in range(nl)]
    pre_all = {}
    for k in range(nl):
        L = plan.level0 + k
        info = plan.info[k]
        nf, cb = info["n_fluid"], info["n_fluid"] - info["n_cap_fluid"]
        xs = np.unique(np.concatenate([rng.integers(0, nf, n_sample),
                                       rng.integers(cb, nf, n_sample // 2)]))
        prev = sim.get_pdf_prev(k)
        pre = sim.get_pdf_pre(k)
        post = sim.get_pdf(k)
        # (a) the pull, by coordinates
        _, co = otree.decode(look[k].tid[xs], d)
        ext = ext0 << k
        want = np.empty((q, len(xs)))
        want[0] = _take(prev, np.zeros(len(xs), np.int64), xs)
        eq_mask = np.zeros((q, len(xs)), dtype=bool)
        for i in range(1, q):
            y = co - c_lib[i]
            eq = np.zeros(len(xs), bool)
            cp = np.zeros(len(xs), bool)
            wall = np.zeros(len(xs), bool)
            for a in range(d):
                for side, m in ((0, y[:, a] < 0), (1, y[:, a] >= ext[a])):
                    f = face[2 * a + side]
                    if f == "periodic":
                        y[m, a] %= ext[a]
                    elif f == "eq":
                        eq |= m
                    elif f == "copy":
                        cp |= m
                    else:
                        wall |= m
            # a link crossing several faces: EQ over COPY over WALL
            cp &= ~eq
            wall &= ~(eq | cp)
            inb = ~(eq | cp | wall)
            j = np.full(len(xs), -1, np.int64)
            j[inb] = look[k].find(otree.encode(L, y[inb]))
            solid = inb & (j < 0)
            assert not solid.any() or k == nl - 1, "missing neighbour below the finest level"
            row = np.full(len(xs), i, np.int64)
            col = j.copy()
            bb = solid | wall
            row[bb], col[bb] = opp[i], xs[bb]
            col[cp | eq] = xs[cp | eq]
            want[i] = _take(prev, row, col)
            want[i][eq] = feq_in[i]
            eq_mask[i] = eq
        got_pre = _cols(pre, xs)
        exact = ~eq_mask
        assert np.array_equal(got_pre[exact], want[exact]), f"pull differs on level {L}"
        if eq_mask.any():
            assert np.abs(got_pre[eq_mask] - want[eq_mask]).max() < 1e-7
        # (b) the collision in FP64 by the oracle
        expect = ophys.collide(torch.from_numpy(got_pre[to_o]), omega[k], lat).numpy()[perm]
        got_post = _cols(post, xs)
        if precision == "f32":
            rel = float((np.abs(got_post - expect) / np.abs(expect)).max())
            assert rel < 2e-6, (L, rel)
        else:
            assert _f16s_ok(got_post, expect, w_lib, c_lib), f"collision on level {L}"
        _say(f"level {L}: {len(xs)} elements: pull exact, collision within bounds")
        pre_all[k] = pre
        del prev, post
    # (c) the fills of the last synchronisation of each level pair
    gpos = [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)] if d == 3 else \
        [(0, 0), (1, 0), (0, 1), (1, 1)]
    tol_rel = 1e-5 if precision == "f32" else None

    def compare(got, exp, what):
        if precision == "f32":
            rel = float((np.abs(got - exp) / np.abs(exp)).max())
            assert rel < tol_rel, (what, rel)
        else:
            g = np.abs(exp - w_lib[:, None])
            assert (np.abs(got - exp) <= 2.0 ** -10 * g + 5e-6 * np.abs(exp)).all(), what

    for k in range(nl - 1):
        L = plan.level0 + k
        ic, fi = plan.info[k], plan.info[k + 1]
        gff_begin = ic["n_fluid"] + ic["n_gfc_inner"] + ic["n_gfc_outer"]
        gsrc = plan.export(k, "gff_src")                      # [4][n_gff] on level k+1

        def gff_pre(gidx):
            """Oracle's pre-collision GhostFromFiner pdfs (library order)."""
            f_src = np.stack([_cols(pre_all[k + 1], gsrc[m, gidx]) for m in range(4)])
            v = ointerp.fill(torch.from_numpy(f_src[:, to_o]), gpos, (0.5,) * d,
                             omega[k + 1], omega[k], 2.0, lat)
            return v.numpy()[perm]

        if ic["n_gff"]:
            gs = np.unique(rng.integers(0, ic["n_gff"], n_sample))
            exp = ophys.collide(torch.from_numpy(gff_pre(gs)[to_o]), omega[k], lat).numpy()[perm]
            post = sim.get_pdf(k)
            got = _cols(post, gff_begin + gs)
            del post
            compare(got, exp, f"GhostFromFiner level {L}")
        ng = fi["n_gfc_inner"] + fi["n_gfc_outer"]
        if ng:
            hs = np.unique(np.concatenate([rng.integers(0, fi["n_gfc_inner"], n_sample // 2),
                                           rng.integers(0, ng, n_sample // 2)]))
            csrc = plan.export(k + 1, "gfc_src")[:, hs]        # [4][m] on level k
            _, cf = otree.decode(look[k + 1].tid[fi["n_fluid"] + hs], d)
            sgn = 2 * (cf & 1) - 1
            # pre-collision pdfs of the coarse sources: fluid, or GhostFromFiner
            # ghosts filled from the fine level's pre-collision pdfs
            f_src = np.empty((4, q, len(hs)))
            for m in range(4):
                s = csrc[m]
                fl = s < ic["n_fluid"]
                assert (fl | (s >= gff_begin)).all()
                if fl.any():
                    f_src[m][:, fl] = _cols(pre_all[k], s[fl])
                if (~fl).any():
                    f_src[m][:, ~fl] = gff_pre(s[~fl] - gff_begin)
            exp = np.empty((q, len(hs)))
            codes = ((sgn + 1) // 2) @ (1 << np.arange(d))
            for oc in np.unique(codes):
                m = codes == oc
                s = sgn[np.where(m)[0][0]]
                if d == 3:
                    pos = [(0, 0, 0), (s[0], s[1], 0), (s[0], 0, s[2]), (0, s[1], s[2])]
                else:
                    pos = [(0, 0), (s[0], 0), (0, s[1]), (s[0], s[1])]
                v = ointerp.fill(torch.from_numpy(f_src[:, to_o][:, :, m]), pos,
                                 tuple(0.25 * float(t) for t in s), omega[k], omega[k + 1],
                                 0.5, lat)
                exp[:, m] = ophys.collide(v, omega[k + 1], lat).numpy()[perm]
            post = sim.get_pdf(k + 1)
            got = _cols(post, fi["n_fluid"] + hs)
            del post
            compare(got, exp, f"GhostFromCoarser level {L + 1}")
        _say(f"fills between levels {L} and {L + 1} within bounds")


def _sphere_case(D, n_levels, precision, warm):
    import paper_1601_06984_amd as M
    uin = [0.04, 0.0, 0.0]
    spec = W.sphere_channel_mesh(D, n_levels, outlet="eq")
    tau_f = 0.5 + 3.0 * uin[0] * D / 100.0
    tau0 = 0.5 + (tau_f - 0.5) / float(1 << (n_levels - 1))
    plan = M.Plan.from_spec(spec)
    sim = M.Sim(plan, precision, tau0, u_in=uin)
    sim.tau0 = tau0
    for k in range(plan.n_levels):
        rho, u = _device_fields(plan, k, spec.box_extent, uin[0], sim.device)
        sim.init(k, rho, u, None)
        del rho, u
    sim.fill_ghosts()
    sim.inputs = {}
    sim.step(warm)
    sim.step(1)
    assert sim.status() == 0
    return spec, plan, sim, uin


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["f32", "f16s"])
def test_sphere3_every_level_one_coarse_step(precision):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    _say(f"sphere channel D=24, 3 levels, {precision}: pull, collision and fills per level")
    spec, plan, sim, uin = _sphere_case(24, 3, precision, warm=2)
    _check_levels(spec, plan, sim, precision, uin, n_sample=30000)


@pytest.mark.timeout(800)
def test_sphere4_every_level_one_coarse_step_f16s():
    """The bench's default workload (449M elements, FP16-shift storage)."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    _say("sphere channel D=128, 4 levels, f16s: pull, collision and fills per level")
    spec, plan, sim, uin = _sphere_case(128, 4, "f16s", warm=1)
    _check_levels(spec, plan, sim, "f16s", uin, n_sample=30000)
