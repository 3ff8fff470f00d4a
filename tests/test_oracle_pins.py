"""Pins of the FP64 oracle against facts the paper and geometry fix.

None of these checks re-types the oracle's own formulas: they use hand
derivations, closed forms of special cases, brute-force algorithms that share
no step with Siddon's method (per-voxel chords, face clipping, fine-step
integration), invariances of the line integral, and finite differences.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers

def _random_ray_through(rng, lo, hi, margin=5.0):
    """Endpoints well outside the box whose segment passes near its centre."""
    c = 0.5 * (np.asarray(lo) + np.asarray(hi))
    ext = np.asarray(hi) - np.asarray(lo)
    target = c + rng.uniform(-0.6, 0.6, 3) * ext
    direction = rng.normal(size=3)
    direction /= np.linalg.norm(direction)
    r = np.linalg.norm(ext) + margin
    return target - r * direction, target + r * direction


# ---------------------------------------------------------------- hand cases

def test_hand_derived_cases():
    """Worked examples derived by hand from Eq. 2 (tests/golden/hand_cases.json)."""
    with open(os.path.join(GOLDEN, "hand_cases.json")) as f:
        g = json.load(f)
    grid = oracle.Grid(np.array(g["volume"]), g["spacing"], g["origin"])
    for case in g["cases"]:
        E, cnt, _ = oracle.trace_rays(grid, np.array([case["s"]]), np.array([case["p"]]))
        assert E[0] == pytest.approx(case["E"], rel=1e-13, abs=1e-13), case["name"]
        assert cnt[0] == case["segments"], case["name"]


# ---------------------------------------------------------------- geometry

def test_geometry_special_poses():
    """Closed forms of the pose convention at special angles (Sec. 2.4 reading)."""
    sdd = 1000.0
    rho = sdd / 2
    # identity pose: source on +x at rho, detector centre on -x at rho
    s, p = oracle.ray_endpoints([0, 0, 0, 0, 0, 0, sdd], 2, 2, 1.0, 1.0, 1, 1)
    np.testing.assert_allclose(s, [rho, 0, 0], atol=1e-12)
    # pixel (1,1) of a 2x2 detector sits at (u, v) = (0.5, 0.5) pitch
    np.testing.assert_allclose(p, [-rho, 0.5, 0.5], atol=1e-12)
    # azimuth theta = pi/2 turns the source onto +y
    s, _ = oracle.ray_endpoints([math.pi / 2, 0, 0, 0, 0, 0, sdd], 1, 1, 1.0, 1.0, 0, 0)
    np.testing.assert_allclose(s, [0, rho, 0], atol=1e-9)
    # phi = pi/2 turns the source onto -z
    s, _ = oracle.ray_endpoints([0, math.pi / 2, 0, 0, 0, 0, sdd], 1, 1, 1.0, 1.0, 0, 0)
    np.testing.assert_allclose(s, [0, 0, -rho], atol=1e-9)
    # gamma = pi/2 rolls the detector about the principal axis: u -> v
    _, p = oracle.ray_endpoints([0, 0, math.pi / 2, 0, 0, 0, sdd], 1, 3, 2.0, 2.0, 0, 2)
    np.testing.assert_allclose(p, [-rho, 0, 2.0], atol=1e-9)
    # two angles fix the order of the factors: with phi = gamma = pi/2,
    # R e_x = Ry(pi/2) Rx(pi/2) e_x = -e_z and R e_y = Ry(pi/2) e_z = +e_x,
    # so pixel (0, 2) of a 1 x 3 detector at pitch 2 (u = 2) sits at (2, 0, rho)
    _, p = oracle.ray_endpoints([0, math.pi / 2, math.pi / 2, 0, 0, 0, sdd], 1, 3, 2.0, 2.0, 0, 2)
    np.testing.assert_allclose(p, [2.0, 0, rho], atol=1e-9)
    # and with theta = phi = pi/2 the source sits at R e_x rho = Rz(pi/2)(-e_z) rho
    s, _ = oracle.ray_endpoints([math.pi / 2, math.pi / 2, 0, 0, 0, 0, sdd], 1, 1, 1.0, 1.0, 0, 0)
    np.testing.assert_allclose(s, [0, 0, -rho], atol=1e-9)
    # translation moves source and detector together
    s, p = oracle.ray_endpoints([0, 0, 0, 1, 2, 3, sdd], 1, 1, 1.0, 1.0, 0, 0)
    np.testing.assert_allclose(s, [rho + 1, 2, 3], atol=1e-12)
    np.testing.assert_allclose(p, [-rho + 1, 2, 3], atol=1e-12)


def test_geometry_invariants_random_poses():
    """Source-detector distance, pixel pitch and orthogonality for any pose."""
    rng = np.random.default_rng(5)
    H, W, dx, dy = 5, 7, 1.3, 0.9
    for _ in range(20):
        pose = np.concatenate([rng.uniform(-3, 3, 3), rng.uniform(-50, 50, 3), [rng.uniform(500, 1500)]])
        s, p00 = oracle.ray_endpoints(pose, H, W, dx, dy, 0, 0)
        _, p01 = oracle.ray_endpoints(pose, H, W, dx, dy, 0, 1)
        _, p10 = oracle.ray_endpoints(pose, H, W, dx, dy, 1, 0)
        # odd detector: pixel (2, 3) is the centre, at distance sdd from s
        _, pc = oracle.ray_endpoints(pose, H, W, dx, dy, 2, 3)
        assert np.linalg.norm(pc - s) == pytest.approx(pose[6], rel=1e-12)
        # source and detector centre are symmetric about the translation
        np.testing.assert_allclose(0.5 * (s + pc), pose[3:6], atol=1e-9)
        eu, ev = p01 - p00, p10 - p00
        assert np.linalg.norm(eu) == pytest.approx(dx, rel=1e-12)
        assert np.linalg.norm(ev) == pytest.approx(dy, rel=1e-12)
        axis = s - pc
        assert abs(np.dot(eu, ev)) < 1e-9
        assert abs(np.dot(eu, axis)) < 1e-7
        assert abs(np.dot(ev, axis)) < 1e-7


def test_endpoint_derivatives_vs_central_differences():
    rng = np.random.default_rng(6)
    H, W, dx, dy = 9, 8, 1.4, 1.1
    for _ in range(10):
        pose = np.concatenate([rng.uniform(-1, 1, 3), rng.uniform(-30, 30, 3), [1020.0]])
        h, w = rng.integers(0, H), rng.integers(0, W)
        ds, dp = oracle.ray_endpoint_derivs(pose, H, W, dx, dy, h, w)
        for j in range(7):
            e = 1e-6
            pp, pm = pose.copy(), pose.copy()
            pp[j] += e
            pm[j] -= e
            sp, ppx = oracle.ray_endpoints(pp, H, W, dx, dy, h, w)
            sm, pmx = oracle.ray_endpoints(pm, H, W, dx, dy, h, w)
            np.testing.assert_allclose(ds[:, j], (sp - sm) / (2 * e), atol=1e-6, rtol=1e-7)
            np.testing.assert_allclose(dp[:, j], (ppx - pmx) / (2 * e), atol=1e-6, rtol=1e-7)


# ---------------------------------------------------------------- E(R)

@pytest.mark.parametrize("dims,spacing", [((4, 5, 6), (1.0, 0.7, 2.5)),
                                          ((64, 64, 64), (1.0, 1.0, 1.0)),
                                          ((3, 1, 7), (2.0, 3.0, 0.5))])
def test_uniform_box_equals_mu_times_chord(dims, spacing):
    """Eq. 1 on a constant volume: E = mu x chord length through the box."""
    rng = np.random.default_rng(1)
    mu = 0.37
    vol = np.full(dims, mu)
    grid = oracle.Grid(vol, spacing)
    lo, hi = grid.origin, grid.origin + np.asarray(dims) * np.asarray(spacing)
    src, dst = zip(*[_random_ray_through(rng, lo, hi) for _ in range(200)])
    E, cnt, _ = oracle.trace_rays(grid, np.array(src), np.array(dst))
    chords = np.array([brute.chord_face_clip(s, p, lo, hi) for s, p in zip(src, dst)])
    np.testing.assert_allclose(E, mu * chords, rtol=1e-12, atol=1e-12)
    assert (E > 0).sum() > 100


def test_axis_aligned_central_ray_is_exact():
    """An axis-aligned ray through a uniform box sees exactly n_c dC mu."""
    dims, spacing = (10, 12, 14), (0.7, 0.9, 2.5)
    grid = oracle.Grid(np.full(dims, 2.0), spacing)
    for c in range(3):
        s = np.array([0.1, 0.2, 0.3])
        p = s.copy()
        s[c], p[c] = -1000.0, 1000.0
        E, cnt, _ = oracle.trace_rays(grid, s[None], p[None])
        assert E[0] == pytest.approx(2.0 * dims[c] * spacing[c], rel=1e-13)
        assert cnt[0] == dims[c]


@pytest.mark.parametrize("seed", range(6))
def test_per_voxel_brute_force(seed):
    """Arbitrary rays through small random volumes: E equals the sum over
    voxels of attenuation x chord through each voxel box, and the number of
    positive-length segments equals the number of voxels with a chord."""
    rng = np.random.default_rng(100 + seed)
    dims = tuple(int(v) for v in rng.integers(1, 8, 3))
    spacing = rng.uniform(0.5, 3.0, 3)
    origin = rng.uniform(-5, 5, 3)
    vol = rng.uniform(0, 2, dims)
    grid = oracle.Grid(vol, spacing, origin)
    lo, hi = origin, origin + np.asarray(dims) * spacing
    n = 60
    src, dst = zip(*[_random_ray_through(rng, lo, hi) for _ in range(n)])
    # a few rays that start or end inside the volume (clamped bounds)
    for _ in range(10):
        a = lo + rng.uniform(0.1, 0.9, 3) * (hi - lo)
        b = a + rng.normal(size=3) * 20
        src, dst = src + (a,), dst + (b,)
    E, cnt, _ = oracle.trace_rays(grid, np.array(src), np.array(dst))
    for r in range(len(src)):
        ref, nvox = brute.per_voxel_sum(vol, spacing, origin, src[r], dst[r])
        assert E[r] == pytest.approx(ref, rel=1e-11, abs=1e-11)
        assert cnt[r] == nvox


def test_fine_step_axis_aligned():
    """Axis-aligned rays whose Riemann samples avoid every plane: exact."""
    rng = np.random.default_rng(3)
    dims, spacing = (6, 5, 4), (1.0, 1.0, 1.0)
    origin = (0.0, 0.0, 0.0)
    vol = rng.uniform(0, 3, dims)
    grid = oracle.Grid(vol, spacing, origin)
    for c in range(3):
        for _ in range(5):
            s = rng.uniform(0.05, 0.95, 3) * np.asarray(dims)
            s = np.floor(s) + 0.5 + rng.uniform(-0.3, 0.3, 3)
            p = s.copy()
            s[c], p[c] = -2.0, dims[c] + 2.0           # length dims+4, integer mm
            n_steps = int(round((p[c] - s[c]) * 8))      # 8 samples per voxel
            ref = brute.fine_step_integral(vol, spacing, origin, s, p, n_steps)
            E, _, _ = oracle.trace_rays(grid, s[None], p[None])
            assert E[0] == pytest.approx(ref, rel=1e-12)


def test_invariances():
    """Linearity in V, direction reversal, axis permutation and integer-voxel
    translation leave the line integral unchanged (Eq. 1)."""
    rng = np.random.default_rng(4)
    dims, spacing = (5, 6, 7), np.array([0.8, 1.1, 1.7])
    V1, V2 = rng.uniform(0, 1, dims), rng.uniform(0, 1, dims)
    g1, g2 = oracle.Grid(V1, spacing), oracle.Grid(V2, spacing)
    g12 = oracle.Grid(2.5 * V1 - 0.5 * V2, spacing)
    lo, hi = g1.origin, g1.origin + np.asarray(dims) * spacing
    src, dst = map(np.array, zip(*[_random_ray_through(rng, lo, hi) for _ in range(50)]))
    E1, c1, _ = oracle.trace_rays(g1, src, dst)
    E2, _, _ = oracle.trace_rays(g2, src, dst)
    E12, _, _ = oracle.trace_rays(g12, src, dst)
    np.testing.assert_allclose(E12, 2.5 * E1 - 0.5 * E2, rtol=1e-12, atol=1e-12)
    Er, cr, _ = oracle.trace_rays(g1, dst, src)
    np.testing.assert_allclose(Er, E1, rtol=1e-12, atol=1e-12)
    assert np.array_equal(cr, c1)
    # permute axes (x, y, z) -> (z, x, y)
    perm = (2, 0, 1)
    gp = oracle.Grid(np.transpose(V1, perm), spacing[list(perm)], g1.origin[list(perm)])
    Ep, _, _ = oracle.trace_rays(gp, src[:, perm], dst[:, perm])
    np.testing.assert_allclose(Ep, E1, rtol=1e-12, atol=1e-12)
    # shifting the grid by whole voxels and the rays by the same amount
    shift = np.array([2, -1, 3]) * spacing
    gs = oracle.Grid(V1, spacing, g1.origin + shift)
    Es, _, _ = oracle.trace_rays(gs, src + shift, dst + shift)
    np.testing.assert_allclose(Es, E1, rtol=1e-10, atol=1e-10)


def test_render_matches_ray_endpoints(small_phantom):
    """render() equals tracing the rays built from ray_endpoints()."""
    ph = small_phantom
    grid = oracle.Grid(ph.volume, ph.spacing, ph.origin)
    pose = np.array([0.2, -0.1, 0.3, 3.0, -2.0, 1.0, 1000.0])
    H, W = 6, 5
    img, cnt, _ = oracle.render(grid, pose, H, W, 2.0, 2.0)
    src, dst = [], []
    for h in range(H):
        for w in range(W):
            s, p = oracle.ray_endpoints(pose, H, W, 2.0, 2.0, h, w)
            src.append(s)
            dst.append(p)
    E, c, _ = oracle.trace_rays(grid, np.array(src), np.array(dst))
    np.testing.assert_array_equal(img.ravel(), E)
    np.testing.assert_array_equal(cnt.ravel(), c)


def test_render_row_window(small_phantom):
    ph = small_phantom
    grid = oracle.Grid(ph.volume, ph.spacing, ph.origin)
    pose = np.array([0.1, 0.2, -0.1, 1.0, 2.0, -3.0, 1000.0])
    full, _, _ = oracle.render(grid, pose, 8, 8, 2.0, 2.0)
    part, _, _ = oracle.render(grid, pose, 8, 8, 2.0, 2.0, rows=(3, 6))
    np.testing.assert_array_equal(part[0, 3:6], full[0, 3:6])
    assert not part[0, :3].any() and not part[0, 6:].any()


# ---------------------------------------------------------------- derivatives

def test_ray_endpoint_gradient_vs_central_differences():
    """Frozen-index d E/d s and d E/d p against FP64 central differences on
    rays whose voxel sequence does not change within the step."""
    rng = np.random.default_rng(7)
    dims, spacing = (6, 7, 5), np.array([1.0, 0.8, 1.6])
    vol = rng.uniform(0, 2, dims)
    grid = oracle.Grid(vol, spacing)
    lo, hi = grid.origin, grid.origin + np.asarray(dims) * spacing
    src, dst = map(np.array, zip(*[_random_ray_through(rng, lo, hi) for _ in range(40)]))
    E, gs, gp = oracle.trace_rays_grad(grid, src, dst)
    E0, _, h0 = oracle.trace_rays(grid, src, dst)
    np.testing.assert_allclose(E, E0, rtol=1e-13, atol=1e-13)
    e = 1e-6
    checked = 0
    for which, grad in (("s", gs), ("p", gp)):
        for c in range(3):
            sp, sm, dp_, dm = src.copy(), src.copy(), dst.copy(), dst.copy()
            if which == "s":
                sp[:, c] += e
                sm[:, c] -= e
            else:
                dp_[:, c] += e
                dm[:, c] -= e
            Ep, _, hp = oracle.trace_rays(grid, sp, dp_)
            Em, _, hm = oracle.trace_rays(grid, sm, dm)
            ok = (hp == h0) & (hm == h0) & (E0 > 0)
            fd = (Ep - Em) / (2 * e)
            np.testing.assert_allclose(grad[ok, c], fd[ok], rtol=1e-5, atol=1e-6)
            checked += ok.sum()
    assert checked > 150


def test_translation_along_ray_and_closed_form():
    """Moving s and p together along the ray leaves E unchanged, so
    sum_c d_c dE/dt_c = 0 for every ray with both ends outside the volume;
    and a pure translation derivative is dE/ds + dE/dp."""
    rng = np.random.default_rng(8)
    dims, spacing = (7, 6, 5), np.array([1.2, 0.9, 1.5])
    vol = rng.uniform(0, 2, dims)
    grid = oracle.Grid(vol, spacing)
    lo, hi = grid.origin, grid.origin + np.asarray(dims) * spacing
    src, dst = map(np.array, zip(*[_random_ray_through(rng, lo, hi) for _ in range(40)]))
    E, gs, gp = oracle.trace_rays_grad(grid, src, dst)
    gt = gs + gp
    d = dst - src
    along = (gt * d).sum(axis=1)
    scale = np.abs(gt).sum(axis=1) * np.linalg.norm(d, axis=1) + 1e-30
    assert np.all(np.abs(along) <= 1e-10 * scale)


def test_render_jacobian_vs_central_differences(small_phantom):
    """Pose Jacobian of whole images against FP64 central differences on the
    pixels whose voxel sequence is unchanged by the step (kink-free)."""
    ph = small_phantom
    grid = oracle.Grid(ph.volume, ph.spacing, ph.origin)
    rng = np.random.default_rng(9)
    H = W = 16
    for _ in range(2):
        pose = np.concatenate([rng.uniform(-0.39, 0.39, 3), rng.uniform(-10, 10, 3), [1000.0]])
        img, jac = oracle.render_jacobian(grid, pose, H, W, 8.0, 8.0)
        ref, _, _ = oracle.render(grid, pose, H, W, 8.0, 8.0)
        np.testing.assert_allclose(img, ref, rtol=1e-13, atol=1e-13)
        # dE/dSDD is ~1e-2, so its step is larger to keep rounding below 1e-6
        steps = [1e-7] * 3 + [1e-6] * 3 + [1e-3]
        fd, ok = oracle.render_fd(grid, pose, H, W, 8.0, 8.0, steps)
        for j in range(7):
            m = ok[:, :, j]
            assert m.sum() > 0.3 * H * W
            scale = np.abs(jac[0, :, :, j]).max() + 1e-30
            err = np.abs(jac[0, :, :, j][m] - fd[:, :, j][m]).max() / scale
            assert err < 1e-6, (j, err)


def test_detector_jacobian_vs_central_differences(small_phantom):
    """d image / d (delta_x, delta_y, offset_u, offset_v) against FP64 central
    differences of render() in each detector parameter, on pixels whose voxel
    sequence does not change, at a non-zero principal-point offset."""
    ph = small_phantom
    grid = oracle.Grid(ph.volume, ph.spacing, ph.origin)
    pose = np.array([0.2, -0.15, 0.1, 2.0, -3.0, 1.0, 1000.0])
    H, W, dx, dy, ou, ov = 15, 17, 4.0, 3.5, 1.3, -0.7
    img, jac = oracle.render_detector_jacobian(grid, pose, H, W, dx, dy, offset=(ou, ov))
    ref, _, h0 = oracle.render(grid, pose, H, W, dx, dy, offset=(ou, ov))
    np.testing.assert_allclose(img, ref, rtol=1e-13, atol=1e-13)
    e = 1e-6
    base = np.array([dx, dy, ou, ov])
    for j in range(4):
        a, b = base.copy(), base.copy()
        a[j] += e
        b[j] -= e
        ip, _, hp = oracle.render(grid, pose, H, W, a[0], a[1], offset=(a[2], a[3]))
        im, _, hm = oracle.render(grid, pose, H, W, b[0], b[1], offset=(b[2], b[3]))
        fd = (ip - im)[0] / (2 * e)
        ok = ((hp == h0) & (hm == h0))[0]
        assert ok.mean() > 0.3
        scale = np.abs(jac[0, :, :, j]).max()
        assert np.abs(jac[0, :, :, j][ok] - fd[ok]).max() < 1e-6 * scale, j
    # the centre column / row does not move with the pitch
    np.testing.assert_allclose(jac[0, :, W // 2, 0], 0.0, atol=1e-9)
    np.testing.assert_allclose(jac[0, H // 2, :, 1], 0.0, atol=1e-9)


def test_offset_by_whole_pixels_shifts_the_image(small_phantom):
    """A principal-point offset of k pixel pitches renders the same rays as
    the pixels k columns (rows) further on: the image shifts by k."""
    ph = small_phantom
    grid = oracle.Grid(ph.volume, ph.spacing, ph.origin)
    pose = np.array([-0.1, 0.25, 0.3, 1.0, 2.0, -1.5, 1000.0])
    H, W, dx, dy = 12, 14, 2.5, 3.0
    base, _, _ = oracle.render(grid, pose, H, W, dx, dy)
    right, _, _ = oracle.render(grid, pose, H, W, dx, dy, offset=(3 * dx, 0.0))
    np.testing.assert_allclose(right[0, :, :W - 3], base[0, :, 3:], rtol=1e-12, atol=1e-12)
    up, _, _ = oracle.render(grid, pose, H, W, dx, dy, offset=(0.0, -2 * dy))
    np.testing.assert_allclose(up[0, 2:, :], base[0, :H - 2, :], rtol=1e-12, atol=1e-12)
    assert np.abs(right[0] - base[0]).max() > 1e-3      # the shift is not trivial


# ---------------------------------------------------------------- ZNCC

def test_zncc_closed_forms():
    rng = np.random.default_rng(10)
    T = rng.uniform(0, 5, (13, 11))
    assert oracle.zncc(T, T) == pytest.approx(1.0, abs=1e-14)
    assert oracle.zncc(3.0 * T + 7.0, T) == pytest.approx(1.0, abs=1e-14)
    assert oracle.zncc(-T, T) == pytest.approx(-1.0, abs=1e-14)
    # equals Pearson's correlation coefficient
    I = rng.uniform(0, 5, (13, 11))
    assert oracle.zncc(I, T) == pytest.approx(np.corrcoef(I.ravel(), T.ravel())[0, 1], abs=1e-14)
    # hand example: I = (1, 2, 3), T = (1, 3, 2): r = 1/2
    assert oracle.zncc([1.0, 2.0, 3.0], [1.0, 3.0, 2.0]) == pytest.approx(0.5, abs=1e-15)


def test_zncc_gradient_vs_central_differences():
    rng = np.random.default_rng(11)
    I, T = rng.uniform(0, 5, 50), rng.uniform(0, 5, 50)
    z, g = oracle.zncc_grad(I, T)
    e = 1e-6
    fd = np.zeros_like(I)
    for i in range(I.size):
        a, b = I.copy(), I.copy()
        a[i] += e
        b[i] -= e
        fd[i] = (oracle.zncc(a, T) - oracle.zncc(b, T)) / (2 * e)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)
    # the gradient is orthogonal to constant shifts and to I - mean(I)
    assert abs(g.sum()) < 1e-12
    assert abs(np.dot(g, I - I.mean())) < 1e-12


# ---------------------------------------------------------------- L2

def test_l2_closed_forms():
    rng = np.random.default_rng(13)
    T = rng.uniform(0, 5, (9, 7))
    assert oracle.l2(T, T) == 0.0
    # constant images: (a - b)^2
    assert oracle.l2(np.full(12, 3.5), np.full(12, 1.25)) == pytest.approx(2.25 ** 2, abs=1e-15)
    # hand example: I = (1, 2, 3), T = (1, 3, 5): (0 + 1 + 4) / 3
    assert oracle.l2([1.0, 2.0, 3.0], [1.0, 3.0, 5.0]) == pytest.approx(5.0 / 3.0, abs=1e-15)
    I = rng.uniform(0, 5, (9, 7))
    # symmetric, shift invariant, quadratic in a common scale
    assert oracle.l2(I, T) == pytest.approx(oracle.l2(T, I), rel=1e-15)
    assert oracle.l2(I + 4.0, T + 4.0) == pytest.approx(oracle.l2(I, T), rel=1e-12)
    assert oracle.l2(3.0 * I, 3.0 * T) == pytest.approx(9.0 * oracle.l2(I, T), rel=1e-13)
    # a mean, not a sum: tiling the pair leaves it unchanged
    assert oracle.l2(np.tile(I, 3), np.tile(T, 3)) == pytest.approx(oracle.l2(I, T), rel=1e-13)


def test_l2_gradient_vs_central_differences():
    rng = np.random.default_rng(14)
    I, T = rng.uniform(0, 5, 40), rng.uniform(0, 5, 40)
    v, g = oracle.l2_grad(I, T)
    e = 1e-5
    fd = np.zeros_like(I)
    for i in range(I.size):
        a, b = I.copy(), I.copy()
        a[i] += e
        b[i] -= e
        fd[i] = (oracle.l2(a, T) - oracle.l2(b, T)) / (2 * e)
    np.testing.assert_allclose(g, fd, rtol=1e-7, atol=1e-10)
    # Euler: the loss is homogeneous of degree 2 in (I - T)
    assert np.dot(g, I - T) == pytest.approx(2.0 * v, rel=1e-12)
