"""Plates with holes (Sec. 7.2; reading Q23) on the GPU's general step
against the oracle, and the hole walls against the edge walls."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.helpers import MAX_NORM_FACTOR, max_rel, rel_l2

pytestmark = pytest.mark.gpu

P_, D_, N_ = 0, 1, 2
EDGES = ("xmin", "xmax", "ymin", "ymax")


def _gpu(nx, ny, u0, v0, n, kinds, vals, mask, precision="fp64", lam=0.1, mu=0.05, tau=0.8, scheme="pc", dx=1.0,
         body=(0.0, 0.0), loads=None, samples=None, sample_every=52):
    from paper_2208_13769_amd import lbm

    s = lbm.Solver(nx, ny, dx, precision, scheme, walled=True)
    s.set_material(1.0, lam, mu, tau)
    if any(body):
        s.set_body_force(np.array(body))
    for e, k in enumerate(kinds):
        if k != P_:
            s.set_boundary(e, k, vals[e])
    if mask is not None:
        s.set_mask(mask)
    s.set_fields(u0, v0)
    series = []
    if loads:
        for k in range(n):
            for e, v in loads(k, s.dt).items():
                s.set_boundary(EDGES.index(e), kinds[EDGES.index(e)], v)
            s.step(1)
            if samples is not None and (k + 1) % sample_every == 0:
                series.append(s.sample(samples[0], samples[1]))
    else:
        s.step(n)
    u, v, P, d, st = s.read()
    sig, E, W = s.read_derived()
    s.close()
    return u, v, P, sig, d, st, series


def _oracle(nx, ny, u0, v0, n, kinds, vals, mask, lam=0.1, mu=0.05, tau=0.8, scheme="pc", dx=1.0,
            body=(0.0, 0.0), loads=None):
    kw = {}
    for e, k, v in zip(EDGES, kinds, vals):
        kw["bc_" + e] = k
        kw["val_" + e] = tuple(v)
    sch = {"pc": O.PC, "explicit": O.EXPLICIT, "extrap": O.EXTRAP}[scheme]
    p = O.Params(nx=nx, ny=ny, dx=dx, lam=lam, mu=mu, tau_over_dt=tau, body=body, scheme=sch, solid=mask, **kw)
    s = O.Solver(p, u0, v0)
    for k in range(n):
        if loads:
            for e, v in loads(k, O.dt(p)).items():
                s.set_boundary_value(e, v)
        s.step(1)
    u, v, P = s.fields()
    sig, E, W = s.derived()
    return u, v, P, sig, s.diagnostics()


def _holes(nx, ny):
    m = np.ones((ny, nx), np.uint8)
    m[6:14, 9:20] = 0
    m[17:21, 4:7] = 0
    return m


@pytest.mark.parametrize("scheme", ["pc", "explicit", "extrap"])
@pytest.mark.parametrize("kinds", [(P_, P_, D_, N_), (N_, D_, N_, N_)])
def test_holes_match_oracle(gpu, kinds, scheme):
    nx, ny, n = 31, 26, 80
    m = _holes(nx, ny)
    rng = np.random.Generator(np.random.PCG64(31))
    u0 = 0.002 * rng.standard_normal((2, ny, nx)) * m[None]
    v0 = 0.002 * rng.standard_normal((2, ny, nx)) * m[None]
    vals = [(0.0, 0.0) if k == P_ else ((0.0001, -0.00005) if k == D_ else (0.0001, 0.0002)) for k in kinds]
    lam = 0.05 if scheme == "extrap" else 0.1
    uo, vo, Po, so, do = _oracle(nx, ny, u0, v0, n, kinds, vals, m, lam=lam, scheme=scheme, body=(2e-5, -1e-5))
    ug, vg, Pg, sg, dg, st, _ = _gpu(nx, ny, u0, v0, n, kinds, vals, m, lam=lam, scheme=scheme, body=(2e-5, -1e-5))
    assert st == 0
    e = [rel_l2(ug, uo), rel_l2(vg, vo), rel_l2(Pg, Po), rel_l2(sg, so)]
    print(f"holes {kinds} {scheme}: rel-L2 u {e[0]:.3e} v {e[1]:.3e} P {e[2]:.3e} sigma {e[3]:.3e}", flush=True)
    assert max(e) < 1e-12
    assert np.abs(ug[:, m == 0]).max() == 0.0 and np.abs(Pg[:, :, m == 0]).max() == 0.0
    assert abs(dg.momentum[0] - do["momentum"][0]) <= 1e-10 * max(1e-30, np.abs(do["momentum"]).max())
    assert abs(dg.energy - do["energy"]) <= 1e-10 * do["energy"]


@pytest.mark.parametrize("scheme", ["pc", "explicit"])
def test_one_node_wide_holes_match_oracle(gpu, scheme):
    """Holes one node wide (a column, a row and a single node): each material
    node beside such a hole sees the hole K of its own gradient, so the two
    nodes on either side see different values (reading Q23)."""
    nx, ny, n = 30, 24, 60
    m = np.ones((ny, nx), np.uint8)
    m[5:15, 7] = 0
    m[18, 12:22] = 0
    m[8, 20] = 0
    rng = np.random.Generator(np.random.PCG64(34))
    u0 = 0.002 * rng.standard_normal((2, ny, nx)) * m[None]
    v0 = 0.002 * rng.standard_normal((2, ny, nx)) * m[None]
    kinds = (N_, D_, D_, N_)
    vals = [(0.0001, 0.0), (0.0, 0.0), (0.0, 0.0), (0.0, 0.0002)]
    uo, vo, Po, so, do = _oracle(nx, ny, u0, v0, n, kinds, vals, m, scheme=scheme)
    ug, vg, Pg, sg, dg, st, _ = _gpu(nx, ny, u0, v0, n, kinds, vals, m, scheme=scheme)
    assert st == 0
    e = [rel_l2(ug, uo), rel_l2(vg, vo), rel_l2(Pg, Po), rel_l2(sg, so)]
    print(f"one-node holes {scheme}: rel-L2 u {e[0]:.3e} v {e[1]:.3e} P {e[2]:.3e} sigma {e[3]:.3e}", flush=True)
    assert max(e) < 1e-12
    assert np.abs(ug[:, m == 0]).max() == 0.0


@pytest.mark.parametrize("precision,scheme,tol", [("fp64", "pc", 1e-12), ("fp64", "explicit", 1e-12),
                                                   ("fp32", "pc", 1e-5), ("fp32u64", "pc", 1e-5),
                                                   ("fp16", "pc", 1e-3)])
@pytest.mark.parametrize("kinds", [(N_, D_, D_, N_), (N_, D_, P_, P_), (P_, P_, D_, N_)])
def test_fused_share_of_the_general_step_matches_oracle(gpu, precision, scheme, tol, kinds):
    """A plate wide enough that the general step hands the fused kernel the
    strips clear of the x walls and of the hole (with x walls: the runs above
    and below the hole in the second strip, and all of the third; periodic
    in x: also the strips whose halo wraps across the edge), next to the 2D
    tiles for the rest, one step or (PC, 32/64-bit storage) two steps at a
    time: against the oracle."""
    nx, ny, n = 700, 160, 41  # paired steps (PC, 32/64-bit storage) and a single one
    m = np.ones((ny, nx), np.uint8)
    m[60:100, 300:400] = 0
    rng = np.random.Generator(np.random.PCG64(35))
    u0 = 0.002 * rng.standard_normal((2, ny, nx)) * m[None]
    v0 = 0.002 * rng.standard_normal((2, ny, nx)) * m[None]
    vals = [(0.0, 0.0) if k == P_ else ((0.0001, 0.0) if e == 0 else (0.0, 2e-4) if k == N_ else (0.0, 0.0))
            for e, k in enumerate(kinds)]
    uo, vo, Po, so, do = _oracle(nx, ny, u0, v0, n, kinds, vals, m, scheme=scheme)
    ug, vg, Pg, sg, dg, st, _ = _gpu(nx, ny, u0, v0, n, kinds, vals, m, precision=precision, scheme=scheme)
    assert st == 0
    e = [rel_l2(ug, uo), rel_l2(vg, vo), rel_l2(Pg, Po)]
    print(f"fused share {precision} {scheme} {kinds}: rel-L2 u {e[0]:.3e} v {e[1]:.3e} P {e[2]:.3e}", flush=True)
    assert max(e[0], e[2]) < tol
    assert np.abs(ug[:, m == 0]).max() == 0.0


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32u64", 1e-5), ("fp16", 1e-3)])
def test_fused_share_without_holes_matches_oracle(gpu, precision, tol):
    """Walls on all four edges and no mask (the loaded block of Sec. 7.1 at
    a size with a fused share): the fused kernel over the strips and rows
    clear of the walls, the 2D tiles for one tile column and row at each
    wall, paired and single steps, against the oracle."""
    nx, ny, n = 700, 160, 41
    rng = np.random.Generator(np.random.PCG64(36))
    u0 = 0.002 * rng.standard_normal((2, ny, nx))
    v0 = 0.002 * rng.standard_normal((2, ny, nx))
    kinds = (N_, D_, D_, N_)
    vals = [(0.0, 0.0), (0.0001, 0.0), (0.0, 0.0), (0.0, 2e-4)]
    uo, vo, Po, so, do = _oracle(nx, ny, u0, v0, n, kinds, vals, None)
    ug, vg, Pg, sg, dg, st, _ = _gpu(nx, ny, u0, v0, n, kinds, vals, None, precision=precision)
    assert st == 0
    e = [rel_l2(ug, uo), rel_l2(Pg, Po)]
    print(f"fused share, walls only, {precision}: rel-L2 u {e[0]:.3e} P {e[1]:.3e}", flush=True)
    assert max(e) < tol


HOLE_N, HOLE_K = 4096, 5


@pytest.fixture(scope="module")
def hole_plate_4096():
    """The benchmark's plate with a hole (4096 x 4096 nodes, side l = 1, a
    centred hole of 0.4 l, traction walls with 0.02 mu on the top and bottom,
    lam = mu = 1, tau/dt = 0.55), started from a smooth random velocity so
    that every node moves, and the oracle's state after HOLE_K steps."""
    from paper_2208_13769_amd import inputs

    n = HOLE_N
    h = int(round(0.4 * n))
    a = (n - h) // 2
    m = np.ones((n, n), np.uint8)
    m[a:a + h, a:a + h] = 0
    u0, v0 = inputs.filtered_random_velocity(n, n, 24.0, 41, 1e-3)
    v0 *= m[None]
    kinds = (N_, N_, N_, N_)
    vals = [(0.0, 0.0), (0.0, 0.0), (0.0, -0.02), (0.0, 0.02)]
    kw = {}
    for e, k, v in zip(EDGES, kinds, vals):
        kw["bc_" + e] = k
        kw["val_" + e] = tuple(v)
    p = O.Params(nx=n, ny=n, dx=1.0 / n, lam=1.0, mu=1.0, tau_over_dt=0.55, solid=m, **kw)
    ref = O.Solver(p, u0, v0)
    ref.step(HOLE_K)
    uo, vo, Po = ref.fields()
    del ref
    return dict(m=m, u0=u0, v0=v0, kinds=kinds, vals=vals, uo=uo, Po=Po)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32u64", 1e-5), ("fp16", 1e-3)])
def test_hole_plate_4096_matches_oracle(gpu, hole_plate_4096, precision, tol):
    """The benchmark's plate with a hole at its full size, whole fields
    against the oracle after five steps: with 32/64-bit populations two
    pairs of steps (the two-step fused kernel over the strips and rows clear
    of the walls and the hole, its row runs sized to one wave of resident
    blocks, beside two launches of 2D tiles) and a single step; with 16-bit
    storage single steps."""
    from paper_2208_13769_amd import lbm

    c = hole_plate_4096
    n = HOLE_N
    s = lbm.Solver(n, n, 1.0 / n, precision, "pc", walled=True)
    s.set_material(1.0, 1.0, 1.0, 0.55)
    for e, (k, v) in enumerate(zip(c["kinds"], c["vals"])):
        s.set_boundary(e, k, v)
    s.set_mask(c["m"])
    s.set_fields(c["u0"], c["v0"])
    s.step(HOLE_K)
    ug, _, Pg, _, st = s.read()
    s.close()
    assert st == 0
    eu, eP = rel_l2(ug, c["uo"]), rel_l2(Pg, c["Po"])
    mu_, mP = max_rel(ug, c["uo"]), max_rel(Pg, c["Po"])
    print(f"hole plate {n}^2 {precision}, {HOLE_K} steps: rel-L2 u {eu:.3e} P {eP:.3e}; "
          f"max-norm u {mu_:.3e} P {mP:.3e}", flush=True)
    assert max(eu, eP) < tol
    assert max(mu_, mP) < MAX_NORM_FACTOR * tol


def test_plate_with_hole_80x80_matches_oracle(gpu):
    """The plate with a hole of Sec. 7.2 as the paper runs it: side l = 1 on
    80 x 80 nodes (dX = 0.0125), a centred square hole of 0.4 l (32 x 32
    nodes), lam = mu = 1, a traction of 0.1 mu on the top and bottom edges
    applied at t = 0 and removed at t = 1, run to t = 3 (416 steps), sides
    and hole free; tau/dt = 0.55 (reading Q24). Also the paper's one
    number: the plate lengthens by about 18 % (here on the centre line, the
    top edge node against the bottom one, sampled every step)."""
    n, h, T = 80, 32, 0.1
    a = (n - h) // 2
    m = np.ones((n, n), np.uint8)
    m[a:a + h, a:a + h] = 0
    kinds = (N_, N_, N_, N_)
    vals = [(0.0, 0.0)] * 4

    def loads(k, dt):
        f = T if k * dt < 1.0 else 0.0
        return {"ymax": (0.0, f), "ymin": (0.0, -f)}

    z = np.zeros((2, n, n))
    q = (np.array([n // 2, n // 2, a + h]), np.array([n - 1, 0, n // 2]))
    kw = dict(lam=1.0, mu=1.0, tau=0.55, dx=1.0 / n, loads=loads)
    uo, vo, Po, so, _ = _oracle(n, n, z, z.copy(), 416, kinds, vals, m, **kw)
    ug, vg, Pg, sg, dg, st, series = _gpu(n, n, z, z.copy(), 416, kinds, vals, m, samples=q, sample_every=1, **kw)
    assert st == 0
    e = [rel_l2(ug, uo), rel_l2(Pg, Po), rel_l2(sg, so)]
    series = np.array(series)  # [step][node][17]
    length = series[:, 0, 1] - series[:, 1, 1]
    peak = length.max()
    t_peak = (np.argmax(length) + 1) * 3.0 / 416
    print(f"hole 80x80: rel-L2 u {e[0]:.3e} P {e[1]:.3e} sigma {e[2]:.3e}; peak lengthening {peak:.4f} at "
          f"t = {t_peak:.2f}; u1(Q1) min {series[:, 2, 0].min():.4f}", flush=True)
    assert max(e) < 1e-11
    assert 0.16 < peak < 0.20 and 0.9 < t_peak < 1.1


def test_fp32_hole(gpu):
    nx, ny, n = 31, 26, 100
    m = _holes(nx, ny)
    rng = np.random.Generator(np.random.PCG64(32))
    u0 = 0.002 * rng.standard_normal((2, ny, nx)) * m[None]
    v0 = 0.002 * rng.standard_normal((2, ny, nx)) * m[None]
    kinds = (N_, N_, D_, N_)
    vals = [(0.0, 0.0), (0.0, 0.0), (0.0, 0.0), (0.0001, 0.0002)]
    uo, vo, Po, so, _ = _oracle(nx, ny, u0, v0, n, kinds, vals, m)
    for prec in ("fp32", "fp32u64"):
        ug, vg, Pg, sg, dg, st, _ = _gpu(nx, ny, u0, v0, n, kinds, vals, m, precision=prec)
        e = [rel_l2(ug, uo), rel_l2(Pg, Po)]
        print(f"hole {prec}: rel-L2 u {e[0]:.3e} P {e[1]:.3e}", flush=True)
        assert max(e) < 1e-5


def test_row_band_equals_the_fused_walled_strip(gpu):
    """A band of hole rows in a y-periodic plate leaves a strip between two
    traction-free walls: the general step with the mask gives what the
    fused kernel gives for that strip with traction walls."""
    nx, ny, k, n = 96, 40, 4, 60
    rng = np.random.Generator(np.random.PCG64(33))
    u0 = 0.002 * rng.standard_normal((2, ny - k, nx))
    v0 = 0.002 * rng.standard_normal((2, ny - k, nx))
    zero = [(0.0, 0.0)] * 4
    ua, va, Pa, sa, _, st, _ = _gpu(nx, ny - k, u0, v0, n, (P_, P_, N_, N_), zero, None)
    m = np.ones((ny, nx), np.uint8)
    m[ny - k:] = 0
    U = np.zeros((2, ny, nx)); V = np.zeros((2, ny, nx))
    U[:, : ny - k] = u0
    V[:, : ny - k] = v0
    ub, vb, Pb, sb, _, st2, _ = _gpu(nx, ny, U, V, n, (P_, P_, P_, P_), zero, m)
    assert st == 0 and st2 == 0
    assert rel_l2(ub[:, : ny - k], ua) < 1e-13 and rel_l2(Pb[:, :, : ny - k], Pa) < 1e-13


def test_mask_errors(gpu):
    from paper_2208_13769_amd import lbm

    n = 20
    m = np.ones((n, n), np.uint8)
    m[5:9, 5:9] = 0
    s = lbm.Solver(n, n, 1.0, "fp64", "pc")
    with pytest.raises(lbm.LbmError) as e:
        s.set_mask(m)
    assert e.value.status == lbm.LBM_ERR_NOMEM
    s.close()
    s = lbm.Solver(n, n, 1.0, "fp64", "pc", walled=True)
    s.set_material(1.0, 0.1, 0.05, 0.8)
    s.set_boundary(lbm.LBM_EDGE_YMIN, lbm.LBM_BC_NEUMANN_T, (0.0, 0.0))
    bad = m.copy()
    bad[0, 3] = 0  # touches the bottom wall
    with pytest.raises(lbm.LbmError) as e:
        s.set_mask(bad)
    assert e.value.status == lbm.LBM_ERR_ARG
    thin = np.ones((n, n), np.uint8)
    thin[4:10, 3:5] = 0
    thin[4:10, 6:8] = 0  # column 5 is material one node thick
    with pytest.raises(lbm.LbmError) as e:
        s.set_mask(thin)
    assert e.value.status == lbm.LBM_ERR_ARG
    s.set_mask(m)
    with pytest.raises(lbm.LbmError) as e:  # periodicity is fixed once a mask is set
        s.set_boundary(lbm.LBM_EDGE_XMIN, lbm.LBM_BC_NEUMANN_T, (0.0, 0.0))
    assert e.value.status == lbm.LBM_ERR_STATE
    s.set_boundary(lbm.LBM_EDGE_YMAX, lbm.LBM_BC_NEUMANN_T, (0.0, 0.01))  # values may change
    s.set_fields(np.zeros((2, n, n)), np.zeros((2, n, n)))
    with pytest.raises(lbm.LbmError) as e:
        s.set_mask(m)
    assert e.value.status == lbm.LBM_ERR_STATE
    s.close()
