"""GPU fixed-lag SLAM backbone (Sec. III-D) vs the CPU oracle, through the C-ABI.

Bar: the scan matcher is integer work -- best candidate, best and second scores and the ray count
bit-exact; the scan factor is the same FP64 operations on both sides -- equal to the last bit; the
Gauss-Newton window is FP64 with a different elimination order (block recursion vs a dense solve) --
poses within 1e-9 and covariances within 1e-8 relative.
"""
import numpy as np
import pytest
import torch

from envpair import say
from oracle import slam_ref as S
from paper_2603_25834_amd import slam

pytestmark = pytest.mark.gpu

NANG = S.NANG


def _batch(seed, sides, R, W, V, sxy, sh, invalid_p=0.1):
    rng = np.random.default_rng(seed)
    n = len(sides)
    grids = []
    for s in sides:
        g = rng.integers(-300, 150, (s, s)).astype(np.int16)
        for _ in range(max(1, s // 16)):          # walls of strong occupied evidence
            y0, x0 = rng.integers(0, s, 2)
            if rng.random() < 0.5:
                g[y0, x0:x0 + rng.integers(3, 30)] = 880
            else:
                g[y0:y0 + rng.integers(3, 30), x0] = 880
        grids.append(g)
    cell_off = np.concatenate([[0], np.cumsum([s * s for s in sides])[:-1]]).astype(np.int64)
    belief = np.concatenate([g.reshape(-1) for g in grids])
    pose = np.zeros((n, 3), np.int32)
    for r, s in enumerate(sides):
        pose[r, 0] = rng.integers(-2 * 65536, (s + 2) * 65536)     # a few start off the grid
        pose[r, 1] = rng.integers(-2 * 65536, (s + 2) * 65536)
        pose[r, 2] = rng.integers(0, NANG)
    pose[0, 2] = 3                                                  # headings next to the wrap
    if n > 1:
        pose[1, 2] = NANG - 2
    rho = (rng.uniform(0.0, 45.0, (n, R)) * 65536).astype(np.int32)
    rho[rng.random((n, R)) < invalid_p] = -1
    if n > 2:
        rho[2] = -1                                                 # a robot with no returns at all
    a_off = (np.arange(R) * (NANG // R)).astype(np.int32)
    return grids, belief, cell_off, np.array(sides, np.int32), pose, rho, a_off


def _gpu_match(belief, cell_off, side, pose, rho, a_off, W, V, sxy, sh):
    cfg = slam.csm_config(W, V, sxy, sh)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = slam.csm_match(d(belief), d(cell_off), d(side), d(pose), d(rho), d(a_off), cfg)
    torch.cuda.synchronize()
    return out.cpu().numpy(), cfg


@pytest.mark.parametrize("W,V,sxy,sh,R", [(4, 5, 32768, 48, 90), (0, 0, 65536, 16, 64), (8, 8, 20000, 100, 481),
                                          (2, 1, 65536, 0, 360)],
                         ids=["lattice_9x9x11", "single_candidate", "max_lattice", "no_heading_step"])
def test_match_bit_exact(W, V, sxy, sh, R):
    sides = [64, 96, 128, 256, 32, 64, 160, 128, 64, 96]
    grids, belief, cell_off, side, pose, rho, a_off = _batch(W * 31 + V + R, sides, R, W, V, sxy, sh)
    say(f"[slam] csm W={W} V={V} step_xy={sxy} step_h={sh} R={R} robots={len(sides)}")
    got, _ = _gpu_match(belief, cell_off, side, pose, rho, a_off, W, V, sxy, sh)
    trig = S._trig()
    for r in range(len(sides)):
        want = S.csm_match(grids[r], int(pose[r, 0]), int(pose[r, 1]), int(pose[r, 2]), rho[r], a_off, W, V, sxy, sh,
                           trig)
        assert tuple(int(v) for v in got[r]) == want, (r, got[r], want)


@pytest.mark.parametrize("sides,max_side,W,V,R", [([300, 64, 128], None, 4, 5, 360), ([256, 64, 200, 96], 96, 4, 5, 360),
                                                  ([100, 64, 37], None, 4, 5, 360), ([256, 64, 200, 96], 16, 4, 5, 360),
                                                  ([300, 64, 37, 256], 1, 0, 0, 64)],
                         ids=["grid_too_big_for_lds", "bands_below_max_side", "sides_not_multiple_of_8",
                              "many_bands", "one_row_bands_and_global_rows"])
def test_match_staged_and_global_grids(sides, max_side, W, V, R):
    """Grids staged in LDS (the reachable box, in bands of rows when it exceeds the LDS the launch sized
    from max_side; rows padded, sides of any residue) or read from global memory (a box row wider than
    that LDS: with a one-candidate lattice and max_side 1 it holds 128 cells) give the same (exact)
    answers."""
    sxy, sh = 65536, 64
    grids, belief, cell_off, side, pose, rho, a_off = _batch(17 + len(sides), sides, R, W, V, sxy, sh)
    cfg = slam.csm_config(W, V, sxy, sh)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    got = slam.csm_match(d(belief), d(cell_off), d(side), d(pose), d(rho), d(a_off), cfg, max_side=max_side)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    trig = S._trig()
    for r in range(len(sides)):
        want = S.csm_match(grids[r], int(pose[r, 0]), int(pose[r, 1]), int(pose[r, 2]), rho[r], a_off, W, V, sxy, sh,
                           trig)
        assert tuple(int(v) for v in got[r]) == want, (r, got[r], want)


def test_match_far_centres_and_offsets():
    """Staged grids are scored in 32-bit cell arithmetic only when the search centre lies within 2^28
    and every ray offset within 2^29 (Q16); a robot beyond either bound is scored in 64 bits in the same
    launch: a centre far off the grid, ranges near the int32 limit on half the rays, a centre just inside
    the bound, and ordinary robots beside them, all against the oracle."""
    W, V, sxy, sh, R = 4, 5, 65536, 64, 128
    sides = [64, 96, 128, 64, 128, 128, 64]
    grids, belief, cell_off, side, pose, rho, a_off = _batch(91, sides, R, W, V, sxy, sh, invalid_p=0.05)
    pose[0, 0] = (1 << 28) + 5 * 65536                  # centre beyond the bound: 64-bit arithmetic
    pose[1, 1] = -(1 << 29)
    rho[3, ::2] = (1 << 31) - 1 - np.arange(0, R, 2)     # offsets near the int32 limit on half the rays
    pose[4, 0] = (1 << 28) - 65536 - 1                  # centre just inside the bound, far off its grid
    # rays without a return near centres 2^30 (Q16) off the grid in y, and in both axes: such a ray must
    # add nothing even where its placeholder offset would land on the grid
    pose[5] = (10 * 65536, (1 << 30) + 10 * 65536, 100)
    pose[6] = ((1 << 30) + 12 * 65536, (1 << 30) + 9 * 65536, 7000)
    say(f"[slam] csm far centres and offsets R={R} robots={len(sides)}")
    got, _ = _gpu_match(belief, cell_off, side, pose, rho, a_off, W, V, sxy, sh)
    trig = S._trig()
    for r in range(len(sides)):
        want = S.csm_match(grids[r], int(pose[r, 0]), int(pose[r, 1]), int(pose[r, 2]), rho[r], a_off, W, V, sxy, sh,
                           trig)
        assert tuple(int(v) for v in got[r]) == want, (r, got[r], want)
    assert got[3][5] == int(np.sum(rho[3] >= 0))        # the far rays count as used rays


def test_factor_matches_oracle_exactly():
    W, V, sxy, sh, R = 4, 5, 32768, 48, 90
    sides = [64, 96, 128, 256, 32, 64]
    grids, belief, cell_off, side, pose, rho, a_off = _batch(11, sides, R, W, V, sxy, sh)
    got, cfg = _gpu_match(belief, cell_off, side, pose, rho, a_off, W, V, sxy, sh)
    meas, info = slam.csm_factor(torch.from_numpy(got).cuda(), torch.from_numpy(pose).cuda(), cfg, 0.05, 896.0,
                                 0.05, 0.02)
    torch.cuda.synchronize()
    trig = S._trig()
    for r in range(len(sides)):
        # the oracle's factor from the oracle's own match, which the GPU's must equal
        mo = S.csm_match(grids[r], int(pose[r, 0]), int(pose[r, 1]), int(pose[r, 2]), rho[r], a_off, W, V, sxy, sh, trig)
        assert tuple(int(v) for v in got[r]) == mo, r
        z, om = S.scan_factor(*mo, int(pose[r, 0]), int(pose[r, 1]), int(pose[r, 2]), sxy, sh,
                              0.05, 896.0, 0.05, 0.02)
        assert np.array_equal(meas[r].cpu().numpy(), z) and np.array_equal(info[r].cpu().numpy(), om), r


def _windows(n, L, seed):
    rng = np.random.default_rng(seed)
    x0 = np.zeros((n, L, 3))
    prior = np.zeros((n, 6))
    odo = np.zeros((n, max(L - 1, 0), 6))
    scan = np.zeros((n, L, 6))
    for w in range(n):
        t = np.zeros((L, 3))
        t[0] = [rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(-3.1, 3.1)]
        for i in range(1, L):
            th = t[i - 1, 2]
            d, dw = rng.uniform(0.0, 0.25), rng.uniform(-0.4, 0.4)
            t[i] = [t[i - 1, 0] + d * np.cos(th), t[i - 1, 1] + d * np.sin(th), S.wrap(th + dw)]
        for i in range(L - 1):
            c, s = np.cos(t[i, 2]), np.sin(t[i, 2])
            dt = t[i + 1, :2] - t[i, :2]
            odo[w, i, :3] = [c * dt[0] + s * dt[1] + rng.normal(0, 0.01), -s * dt[0] + c * dt[1] + rng.normal(0, 0.01),
                             S.wrap(t[i + 1, 2] - t[i, 2] + rng.normal(0, 0.005))]
            odo[w, i, 3:] = rng.uniform(100, 2500, 3)
        prior[w, :3] = t[0] + rng.normal(0, 0.02, 3)
        prior[w, 3:] = rng.uniform(20, 500, 3)
        has = rng.random(L) < 0.5
        scan[w, has, :3] = t[has] + rng.normal(0, 0.03, (int(has.sum()), 3))
        scan[w, has, 3:] = rng.uniform(5, 400, (int(has.sum()), 3))
        x0[w] = t + rng.normal(0, 0.05, (L, 3))
    scan[:, :, 2] = S.wrap(scan[:, :, 2])
    return x0, prior, odo, scan


@pytest.mark.parametrize("L,iters", [(1, 2), (2, 3), (8, 3), (16, 5), (30, 3), (64, 2), (10, 0)])
def test_fixedlag_matches_oracle(L, iters):
    n = 48
    x0, prior, odo, scan = _windows(n, L, 100 + L)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x, cov = slam.fixedlag_solve(d(x0), d(prior), d(odo) if L > 1 else None, d(scan), iters)
    torch.cuda.synchronize()
    x, cov = x.cpu().numpy(), cov.cpu().numpy()
    worst_x, worst_c = 0.0, 0.0
    for w in range(n):
        xr, Sr = S.fixedlag_solve(x0[w], prior[w], odo[w], scan[w], iters)
        worst_x = max(worst_x, float(np.abs(x[w] - xr).max()))
        worst_c = max(worst_c, float(np.abs(cov[w] - Sr).max() / np.abs(Sr).max()))
    say(f"[slam] fixed-lag L={L} iters={iters}: max |dx| {worst_x:.2e}, max rel dSigma {worst_c:.2e}")
    assert worst_x < 1e-9 and worst_c < 1e-8


def test_full_batch_sampled_and_errors():
    """750 robots of 256^2 grids, 360 rays, the 9 x 9 x 11 lattice: 16 sampled robots against the oracle;
    then the argument checks."""
    from paper_2603_25834_amd import _lib
    W, V, sxy, sh, R = 4, 5, 65536, 64, 360
    sides = [256] * 750
    grids, belief, cell_off, side, pose, rho, a_off = _batch(21, sides, R, W, V, sxy, sh, invalid_p=0.05)
    got, cfg = _gpu_match(belief, cell_off, side, pose, rho, a_off, W, V, sxy, sh)
    trig = S._trig()
    for r in np.random.default_rng(3).choice(750, 16, replace=False):
        want = S.csm_match(grids[r], int(pose[r, 0]), int(pose[r, 1]), int(pose[r, 2]), rho[r], a_off, W, V, sxy, sh,
                           trig)
        assert tuple(int(v) for v in got[r]) == want, r
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    with pytest.raises(_lib.AslamError):
        slam.csm_match(d(belief[:16]), d(cell_off[:1]), d(side[:1]), d(pose[:1]), d(rho[:1]), d(a_off),
                       slam.csm_config(9, 0, 65536, 0))
    with pytest.raises(_lib.AslamError):   # (2V + 1) R > 8192
        slam.csm_match(d(belief[:16]), d(cell_off[:1]), d(side[:1]), d(pose[:1]), d(np.zeros((1, 1000), np.int32)),
                       d(np.zeros(1000, np.int32)), slam.csm_config(1, 8, 65536, 1))


# ------------------------------------------------------------------ weighted map integration

def _integrate_case(seed, sides, R, W, V, sxy, sh, rmax_q, weighted=True, max_side=None):
    grids, belief, cell_off, side, pose, rho, a_off = _batch(seed, sides, R, W, V, sxy, sh)
    trig = S._trig()
    rng = np.random.default_rng(seed + 1)
    match = None
    if weighted:
        # the oracle's own matches, with a few margins moved so that weights span [0, 1]
        match = np.array([S.csm_match(grids[r], int(pose[r, 0]), int(pose[r, 1]), int(pose[r, 2]), rho[r], a_off,
                                      W, V, sxy, sh, trig) for r in range(len(sides))], np.int64)
        for r in range(0, len(sides), 3):
            match[r, 3] = int((match[r, 5]) * 896 * rng.uniform(0.2, 1.0))
            match[r, 4] = int(match[r, 3] * rng.uniform(-0.5, 0.9))
        match = match.astype(np.int32)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    bel = d(belief)
    cfg = slam.csm_config(W, V, sxy, sh)
    coded = slam.csm_integrate(bel, d(cell_off), d(side), d(pose), d(rho), d(a_off), rmax_q, 218, -102, 896,
                               match=None if match is None else d(match), cfg=cfg, l_max=896.0, max_side=max_side)
    torch.cuda.synchronize()
    got = bel.cpu().numpy()
    coded = coded.cpu().numpy()
    for r in range(len(sides)):
        want, nc = S.integrate(grids[r], int(pose[r, 0]), int(pose[r, 1]), int(pose[r, 2]), rho[r], a_off, rmax_q,
                               218, -102, 896, match=None if match is None else match[r], step_xy=sxy, step_h=sh,
                               l_max=896.0)
        s = sides[r]
        o = int(cell_off[r])
        assert np.array_equal(got[o:o + s * s].reshape(s, s), want), r
        assert int(coded[r]) == nc, (r, coded[r], nc)
    return coded


@pytest.mark.parametrize("weighted", [True, False], ids=["weighted", "unweighted"])
def test_integrate_bit_exact(weighted):
    sides = [64, 96, 128, 256, 32, 64, 160, 128, 64, 96]
    say(f"[slam] integrate weighted={weighted} robots={len(sides)}")
    coded = _integrate_case(41, sides, 90, 4, 5, 32768, 48, 30 * 65536, weighted)
    assert (coded > 0).sum() >= 3


def test_integrate_bands_and_max_side():
    """Grids larger than one band of the LDS bitmaps (side 600 with a 64 KB budget; side 300 with the
    bitmaps sized for side 64) give the same exact answers."""
    say("[slam] integrate in bands")
    _integrate_case(43, [600, 64, 128], 120, 2, 2, 65536, 64, 200 * 65536)
    _integrate_case(44, [300, 64, 200, 96], 90, 2, 2, 65536, 64, 120 * 65536, max_side=64)


def test_integrate_many_rays_and_no_count():
    """More rays than the length sort takes (2100 > 2048: rays in their own order), and the call without
    the coded-cell output: same exact grids as the oracle."""
    from paper_2603_25834_amd import _lib
    sides = [64, 96, 48]
    W, V, sxy, sh, R = 1, 0, 65536, 0, 2100
    grids, belief, cell_off, side, pose, rho, a_off = _batch(51, sides, R, W, V, sxy, sh)
    a_off = (np.arange(R) * 21).astype(np.int32)          # headings need not divide the table evenly
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    say(f"[slam] integrate with R={R} rays, with and without the coded-cell output")
    bel = d(belief)
    coded = slam.csm_integrate(bel, d(cell_off), d(side), d(pose), d(rho), d(a_off), 50 * 65536, 218, -102, 896)
    bel2 = d(belief)
    # device copies held by names for the raw call (a temporary could be freed and its memory reused by the
    # next argument before the launch)
    co2, sd2, po2, rh2, ao2 = d(cell_off), d(side), d(pose), d(rho), d(a_off)
    _lib.check(_lib.lib().aslam_csm_integrate(slam.handle().h, slam._p(bel2), slam._p(co2), slam._p(sd2), len(sides),
                                              slam._p(po2), slam._p(rh2), R, slam._p(ao2), 96, 50 * 65536, None, None,
                                              1.0, 218, -102, 896, None, slam._stream()))
    torch.cuda.synchronize()
    got, got2, coded = bel.cpu().numpy(), bel2.cpu().numpy(), coded.cpu().numpy()
    for r, s_ in enumerate(sides):
        want, nc = S.integrate(grids[r], int(pose[r, 0]), int(pose[r, 1]), int(pose[r, 2]), rho[r], a_off, 50 * 65536,
                               218, -102, 896)
        o = int(cell_off[r])
        assert np.array_equal(got[o:o + s_ * s_].reshape(s_, s_), want) and int(coded[r]) == nc, r
        assert np.array_equal(got2[o:o + s_ * s_].reshape(s_, s_), want), r


def test_integrate_full_batch_sampled_and_errors():
    """750 robots of 256^2 grids and 360 rays integrated from the GPU matcher's own output; for 12 sampled
    robots the oracle matches (which the GPU's must equal) drive the oracle's integration; then the
    argument checks."""
    from paper_2603_25834_amd import _lib
    W, V, sxy, sh, R = 4, 5, 65536, 64, 360
    sides = [256] * 750
    grids, belief, cell_off, side, pose, rho, a_off = _batch(23, sides, R, W, V, sxy, sh, invalid_p=0.05)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    cfg = slam.csm_config(W, V, sxy, sh)
    match = slam.csm_match(d(belief), d(cell_off), d(side), d(pose), d(rho), d(a_off), cfg)
    bel = d(belief)
    coded = slam.csm_integrate(bel, d(cell_off), d(side), d(pose), d(rho), d(a_off), 200 * 65536, 218, -102, 896,
                               match=match, cfg=cfg, l_max=896.0)
    torch.cuda.synchronize()
    got, m, coded = bel.cpu().numpy(), match.cpu().numpy(), coded.cpu().numpy()
    trig = S._trig()
    for r in np.random.default_rng(4).choice(750, 12, replace=False):
        # the oracle integrates from its own match, which the GPU's must equal
        mo = S.csm_match(grids[r], int(pose[r, 0]), int(pose[r, 1]), int(pose[r, 2]), rho[r], a_off, W, V, sxy, sh, trig)
        assert tuple(int(v) for v in m[r]) == mo, r
        want, nc = S.integrate(grids[r], int(pose[r, 0]), int(pose[r, 1]), int(pose[r, 2]), rho[r], a_off,
                               200 * 65536, 218, -102, 896, match=mo, step_xy=sxy, step_h=sh, l_max=896.0)
        o = int(cell_off[r])
        assert np.array_equal(got[o:o + 65536].reshape(256, 256), want) and int(coded[r]) == nc, r
    with pytest.raises(_lib.AslamError):   # l_clamp out of range
        slam.csm_integrate(bel, d(cell_off), d(side), d(pose), d(rho), d(a_off), 65536, 218, -102, 0)
    co, sd, po, rh, ao = d(cell_off), d(side), d(pose), d(rho), d(a_off)
    with pytest.raises(_lib.AslamError):   # a match without a config
        _lib.check(_lib.lib().aslam_csm_integrate(slam.handle().h, slam._p(bel), slam._p(co), slam._p(sd), 750,
                                                  slam._p(po), slam._p(rh), R, slam._p(ao), 256, 65536, slam._p(match),
                                                  None, 896.0, 218, -102, 896, None, slam._stream()))
    with pytest.raises(_lib.AslamError):   # no handle
        _lib.check(_lib.lib().aslam_csm_integrate(None, slam._p(bel), slam._p(co), slam._p(sd), 750, slam._p(po),
                                                  slam._p(rh), R, slam._p(ao), 256, 65536, None, None, 896.0, 218,
                                                  -102, 896, None, slam._stream()))


def test_backbone_on_env_state():
    """The four calls in sequence on the state an env reached: 16 robots of 64^2 grids and 180 rays stepped
    20 times on the GPU and by the oracle env (their states agree bit for bit); the GPU backbone runs on the
    GPU env's state and the oracle backbone on the oracle env's -- scan matching of the last scan around the
    estimated pose, the scan factor, the weighted integration from the match, and a 6-pose window whose
    newest pose carries the scan factor."""
    from envpair import Pair
    from oracle import oracle as O
    from paper_2603_25834_amd import _lib
    pr = Pair("small_16x64", 7, steps=20, exec_kw=dict(form=1, threads=256, record_rays=1))
    o = None
    for _ in range(20):
        o = pr.step()
    g = pr.compare(o)
    say("[slam] backbone on the env state of small_16x64 after 20 steps")
    p, n, R = pr.p, pr.n, pr.R
    sides = np.asarray(pr.b.sides, np.int64)
    cell_off = np.concatenate([[0], np.cumsum(sides * sides)[:-1]]).astype(np.int64)
    inv_c16 = np.float32(65536.0 / float(np.float32(p["cell_m"])))
    rmax_q = int(round(float(np.float32(p["r_max_m"])) / float(np.float32(p["cell_m"])) * 65536.0))
    a_off = (np.arange(R) * (S.NANG // R)).astype(np.int32)
    W, V, sxy, sh, L = 3, 4, 65536, 64, 6
    cm, lmax, sig_xy, sig_th = float(p["cell_m"]), 896.0, 0.05, 0.02

    def inputs(est, rho, hitc):
        pose = np.stack([np.rint(est[:, 0].astype(np.float32) * inv_c16), np.rint(est[:, 1].astype(np.float32) * inv_c16),
                         [O.heading_index(float(t)) for t in est[:, 2]]], 1).astype(np.int32)
        return pose, np.where(hitc >= 0, rho, -1).astype(np.int32)

    def window(est, z, om):
        x0 = np.repeat(est.astype(np.float64)[:, None, :], L, 1)
        x0 += 0.01 * np.sin(np.arange(n * L * 3, dtype=np.float64)).reshape(n, L, 3)
        prior = np.concatenate([x0[:, 0], np.full((n, 3), 400.0)], 1)
        odo = np.concatenate([np.zeros((n, L - 1, 3)), np.full((n, L - 1, 3), 2500.0)], 2)
        scan = np.zeros((n, L, 6))
        scan[:, -1, :3], scan[:, -1, 3:] = z, om
        return x0, prior, odo, scan

    # oracle side: the oracle env's state
    orc = pr.orc
    pose_o, rho_o = inputs(orc.est, o.rho_q, o.hit_cell)
    trig = S._trig()
    match_o, z_o, om_o, grid_o, coded_o = [], [], [], [], []
    for r in range(n):
        m = S.csm_match(orc.belief_of(r), int(pose_o[r, 0]), int(pose_o[r, 1]), int(pose_o[r, 2]), rho_o[r], a_off,
                        W, V, sxy, sh, trig)
        z, om = S.scan_factor(*m, int(pose_o[r, 0]), int(pose_o[r, 1]), int(pose_o[r, 2]), sxy, sh, cm, lmax, sig_xy,
                              sig_th)
        gi, nc = S.integrate(orc.belief_of(r), int(pose_o[r, 0]), int(pose_o[r, 1]), int(pose_o[r, 2]), rho_o[r],
                             a_off, rmax_q, 218, -102, 896, match=m, step_xy=sxy, step_h=sh, l_max=lmax)
        match_o.append(m); z_o.append(z); om_o.append(om); grid_o.append(gi); coded_o.append(nc)
    x0o, pro, odo_o, sco = window(orc.est, np.array(z_o), np.array(om_o))
    lag_o = [S.fixedlag_solve(x0o[r], pro[r], odo_o[r], sco[r], 3) for r in range(n)]

    # GPU side: the GPU env's state, through the C-ABI
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    pose_g, rho_g = inputs(g["est"], g["rho"], g["hitc"])
    cfg = slam.csm_config(W, V, sxy, sh)
    bel = pr.env.read(_lib.FIELD_BELIEF)
    CO, SD, PO = d(cell_off), d(sides.astype(np.int32)), d(pose_g)
    match = slam.csm_match(bel, CO, SD, PO, d(rho_g), d(a_off), cfg)
    meas, info = slam.csm_factor(match, PO, cfg, cm, lmax, sig_xy, sig_th)
    coded = slam.csm_integrate(bel, CO, SD, PO, d(rho_g), d(a_off), rmax_q, 218, -102, 896, match=match, cfg=cfg,
                               l_max=lmax)
    x0g, prg, odg, scg = window(g["est"], meas.cpu().numpy(), info.cpu().numpy())
    xg, covg = slam.fixedlag_solve(d(x0g), d(prg), d(odg), d(scg), 3)
    torch.cuda.synchronize()
    match, meas, info = match.cpu().numpy(), meas.cpu().numpy(), info.cpu().numpy()
    bel, coded, xg, covg = bel.cpu().numpy(), coded.cpu().numpy(), xg.cpu().numpy(), covg.cpu().numpy()
    for r in range(n):
        s_, off = int(sides[r]), int(cell_off[r])
        assert tuple(int(v) for v in match[r]) == match_o[r], r
        assert np.array_equal(meas[r], z_o[r]) and np.array_equal(info[r], om_o[r]), r
        assert np.array_equal(bel[off:off + s_ * s_].reshape(s_, s_), grid_o[r]) and int(coded[r]) == coded_o[r], r
        assert np.abs(xg[r] - lag_o[r][0]).max() < 1e-9, r
        assert np.abs(covg[r] - lag_o[r][1]).max() <= 1e-8 * np.abs(lag_o[r][1]).max(), r
    assert sum(coded_o) > 0 and any(w[0] > 0 for w in om_o)


def test_backbone_calls_captured_in_one_graph():
    """Scan matching, the scan factor, the weighted integration and the fixed-lag solve captured in one
    HIP graph (the calls allocate nothing and never synchronise once the handle exists) and replayed
    three times, each replay matching on the grids the previous one integrated into: equal bit for bit
    to the same three rounds launched eagerly."""
    W, V, sxy, sh, R, L = 4, 5, 65536, 64, 360, 8
    sides = [256] * 64
    grids, belief, cell_off, side, pose, rho, a_off = _batch(31, sides, R, W, V, sxy, sh, invalid_p=0.05)
    # grids biased towards occupied evidence, so the best scores are positive and the weights non-zero
    belief = np.clip(belief.astype(np.int32) + 400, -896, 896).astype(np.int16)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    n = len(sides)
    cfg = slam.csm_config(W, V, sxy, sh)
    slam.handle()   # created (allocates) before the capture
    CO, SD, PO, RH, AO = d(cell_off), d(side), d(pose), d(rho), d(a_off)
    rng = np.random.default_rng(5)
    x0 = rng.uniform(1.0, 12.0, (n, 1, 3)) + 0.01 * rng.standard_normal((n, L, 3))
    prior = d(np.concatenate([x0[:, 0], np.full((n, 3), 400.0)], 1))
    odo = d(np.concatenate([np.zeros((n, L - 1, 3)), np.full((n, L - 1, 3), 2500.0)], 2))
    X0 = d(x0)

    def make_state():
        return dict(bel=d(belief), match=torch.empty((n, 6), dtype=torch.int32, device="cuda"),
                    meas=torch.empty((n, 3), dtype=torch.float64, device="cuda"),
                    info=torch.empty((n, 3), dtype=torch.float64, device="cuda"),
                    coded=torch.empty(n, dtype=torch.int32, device="cuda"),
                    scan=torch.zeros((n, L, 6), dtype=torch.float64, device="cuda"),
                    x=torch.empty((n, L, 3), dtype=torch.float64, device="cuda"),
                    cov=torch.empty((n, 3, 3), dtype=torch.float64, device="cuda"))

    def round_(st):
        slam.csm_match(st["bel"], CO, SD, PO, RH, AO, cfg, out=st["match"], max_side=256)
        slam.csm_factor(st["match"], PO, cfg, 0.05, 896.0, 0.05, 0.02, meas=st["meas"], info=st["info"])
        slam.csm_integrate(st["bel"], CO, SD, PO, RH, AO, 200 * 65536, 218, -102, 896, match=st["match"], cfg=cfg,
                           l_max=896.0, coded=st["coded"], max_side=256)
        st["scan"][:, -1, :3].copy_(st["meas"])
        st["scan"][:, -1, 3:].copy_(st["info"])
        slam.fixedlag_solve(X0, prior, odo, st["scan"], 3, x=st["x"], cov=st["cov"])

    eager, graphed = make_state(), make_state()
    round_(graphed)        # warm-up round outside the capture, repeated by the eager side
    round_(eager)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        round_(graphed)
    for k in range(3):
        g.replay()
        round_(eager)
        torch.cuda.synchronize()
        for key in ("bel", "match", "coded", "meas", "info", "x", "cov"):
            assert torch.equal(graphed[key], eager[key]), (k, key)
    # the rounds changed the grids (the integration ran with non-zero weights on every replay)
    assert (graphed["info"][:, 0] > 0).sum().item() > n // 2
    assert not torch.equal(graphed["bel"], d(belief))
