"""Several time steps per launch (temporal blocking) on the GPU.

lb_step_n takes up to four steps per launch (as lb_blocked_steps reports for
the configuration) unless the sum of rho is recorded, a patch is present, a
checkpoint falls inside the launch or the descriptor caps the steps per
launch.  The blocked kernel must give the same bits as launches of the
one-step kernel: the tests below compare the paths bitwise over lattices,
collisions, storage formats, caps of 2 and 3 steps, grid shapes that leave
ragged wavefront strips and segments (of 4, 6 and 8 rows), step counts of
every remainder and chunked calls, with receivers and the source on strip
and segment boundaries and on the periodic seam, and hold the blocked path
to the FP64 oracle bars.
"""
import numpy as np
import pytest

from paper_1704_03172_amd import inputs
from tests.harness import FIELDS, run_gpu, run_oracle
from tests.test_gpu_parity import compare, layered_case

pytestmark = pytest.mark.gpu


def same(a, b):
    assert a["time"] == b["time"]
    np.testing.assert_array_equal(a["traces"], b["traces"])
    for f in FIELDS:
        np.testing.assert_array_equal(a["fields"][f], b["fields"][f])


def both(case, precision, spl=0, **kw):
    one = run_gpu(case, precision, sum_rho=False, steps_per_launch=1)
    two = run_gpu(case, precision, sum_rho=False, steps_per_launch=spl, **kw)
    assert np.abs(one["traces"]).max() > 0
    same(one, two)
    return two


def boundary_receivers(nx, ny):
    """Receivers on the strip edges of every storage format (owned widths
    120 for FP32, 56 for FP64, 224 for FP16 storage), on 3-, 4-, 5-, 6-, 7-
    and 8-row segment edges and on the periodic seam."""
    xs = {0, 1, nx - 1, nx - 2}
    for w in (56, 120, 224):
        for k in range(1, nx // w + 1):
            xs.update({k * w - 1, k * w, k * w + 1})
    ys = {0, 1, ny - 1, ny - 2}
    for h in (3, 4, 5, 6, 7, 8):
        for k in range(1, ny // h + 1):
            ys.update({h * k - 1, h * k})
    xs = sorted(x for x in xs if 0 <= x < nx)
    ys = sorted(y for y in ys if 0 <= y < ny)
    return np.array([(x, y) for y in ys for x in xs[::3]] + [(x, ys[len(ys) // 2]) for x in xs],
                    dtype=np.int32)


SCHEMES = [(5, "bgk", None), (5, "mrt", [1, 1, 1, 1.6, 1.3]), (9, "bgk", None),
           (9, "mrt", [1, 1, 1, 2, 2, 2, 1, 1, 2])]


@pytest.mark.parametrize("precision", ["f32", "f64", "f16s"])
@pytest.mark.parametrize("q,collision,s", SCHEMES)
@pytest.mark.parametrize("spl", [0, 2, 3])
def test_two_step_equals_one_step(precision, q, collision, s, spl):
    case = layered_case(700, 45, q=q, collision=collision, s=s, nsteps=61)
    case["receivers"] = np.concatenate([case["receivers"], boundary_receivers(700, 45)])
    two = both(case, precision, spl=spl)
    if precision != "f16s":
        compare(case, precision, gpu=two)


@pytest.mark.parametrize("precision", ["f32", "f64", "f16s"])
@pytest.mark.parametrize("q", [5, 9])
def test_general_bgk_equals_one_step(precision, q):
    """BGK with tau != 1/2 (the general collision g - omega (g - g^eq); at
    tau = 1/2 every kernel writes it as 2 g^eq - g instead): the blocked
    kernel gives the bits of one step per launch and meets the oracle bars."""
    case = layered_case(400, 37, q=q, collision="bgk", tau=0.8, nsteps=45)
    case["receivers"] = np.concatenate([case["receivers"], boundary_receivers(400, 37)])
    two = both(case, precision)
    if precision != "f16s":
        compare(case, precision, gpu=two)


@pytest.mark.parametrize("nsteps", [2, 3, 4, 5, 6, 7, 8, 9, 30, 31, 32, 33])
def test_step_count_remainders(nsteps):
    """Every remainder of the step count modulo the four steps per launch
    (the last launch of a call takes one step)."""
    case = layered_case(300, 30, nsteps=nsteps, sponge=2)
    case["wavelet"] = 1e3 * case["wavelet"]
    both(case, "f32")


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("nx,ny", [(1, 1), (3, 2), (5, 7), (56, 61), (112, 16), (113, 17), (120, 5),
                                   (121, 9), (224, 3), (2, 300), (1029, 3), (448, 9)])
def test_two_step_shapes(precision, nx, ny):
    rho, jx, jy = inputs.random_fields(nx, ny, seed=nx * 17 + ny)
    rng = np.random.default_rng(nx * ny + 3)
    for q in (5, 9):
        case = {"nx": nx, "ny": ny, "q": q, "collision": "mrt" if q == 9 else "bgk",
                "tau": 0.5, "s": [1, 1, 1, 2, 2, 2, 1, 1, 2][:q],
                "c2": rng.uniform(0.05, 0.45, (ny, nx)), "rho0": rho, "jx0": jx, "jy0": jy,
                "nsteps": 27, "sponge_width": 1 if min(nx, ny) > 4 else 0, "sponge_sigma_max": 0.1,
                "source": (nx - 1, 0), "wavelet": 1e-3 * inputs.ricker_wavelet(28, 0.1),
                "receivers": np.concatenate([np.array([(0, 0), (nx - 1, ny - 1), (nx // 2, ny // 2)],
                                                      dtype=np.int32), boundary_receivers(nx, ny)])}
        two = both(case, precision)
        compare(case, precision, gpu=two, j_floor=True)


# source nodes on strip edges (owned widths 120, 56 and 224), on 5-, 6- and
# 8-row segment edges, on the periodic seam and inside the sponge (where the
# source is added before the sponge factor multiplies the node)
EDGE_SOURCES = [(119, 5), (120, 6), (55, 11), (56, 12), (223, 24), (224, 25), (239, 15), (240, 16),
                (0, 0), (699, 44), (121, 1), (300, 43), (350, 17), (351, 18)]


@pytest.mark.parametrize("precision", ["f32", "f64", "f16s"])
@pytest.mark.parametrize("q,collision,s", [(5, "bgk", None), (5, "mrt", [1, 1, 1, 1.6, 1.3]), (9, "bgk", None)])
def test_source_on_strip_and_segment_edges(precision, q, collision, s):
    """The source row is tested once per row (wave-uniform) in the blocked
    kernel, also where the row is a halo row that a neighbouring wave
    recomputes: every placement gives the bits of one step per launch."""
    if q == 9 and precision == "f16s":
        pytest.skip("D2Q9 with FP16 storage takes one step per launch")
    for k, src in enumerate(EDGE_SOURCES):
        case = layered_case(700, 45, q=q, collision=collision, s=s, nsteps=23, sponge=3)
        case["source"] = src
        case["wavelet"] = 1e2 * case["wavelet"]
        case["receivers"] = np.concatenate([case["receivers"], np.array([src], dtype=np.int32)])
        two = both(case, precision)
        if precision == "f64" and k % 5 == 0:
            compare(case, precision, gpu=two)


@pytest.mark.parametrize("ny", [3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 15, 16, 17, 18, 19, 23, 40])
def test_segment_edges(ny):
    """Grid heights around multiples of the segment heights (ragged last
    segment, a single segment, rows that wrap into the next segment and
    grids shorter than the halo): D2Q5 FP32 BGK with four steps (6-row
    segments, rows loaded six ahead of the walk), D2Q5 FP32 MRT with four
    (6 rows), D2Q5 FP32 with three (6 rows) and two (8 rows), D2Q5 FP64 MRT
    with four (7 rows), D2Q5 FP16 storage with three (5 rows for BGK at
    tau = 1/2, 4 for MRT), D2Q9 BGK FP32
    with three (5 rows), D2Q9 BGK FP64 with four (6 rows), D2Q9 MRT FP32
    with three (3 rows) and two (3 rows) and D2Q9 MRT FP64 with four (5
    rows), so that every
    direction crosses the segment edges."""
    mrt9 = [1, 1, 1, 2, 2, 2, 1, 1, 2]
    mrt5 = [1, 1, 1, 1.6, 1.3]
    for q, coll, s, prec, spl in ((5, "bgk", None, "f32", 0), (5, "mrt", mrt5, "f32", 0), (5, "bgk", None, "f32", 3),
                                  (5, "bgk", None, "f32", 2), (5, "mrt", mrt5, "f64", 0), (5, "bgk", None, "f16s", 0),
                                  (5, "mrt", mrt5, "f16s", 0),
                                  (9, "bgk", None, "f32", 0), (9, "bgk", None, "f64", 0), (9, "mrt", mrt9, "f32", 0),
                                  (9, "mrt", mrt9, "f32", 2), (9, "mrt", mrt9, "f64", 0)):
        case = layered_case(300, ny, q=q, collision=coll, s=s, nsteps=40, sponge=2 if ny > 4 else 0)
        case["receivers"] = np.concatenate([case["receivers"], boundary_receivers(300, ny)])
        two = both(case, prec, spl=spl)
        if prec != "f16s":
            compare(case, prec, gpu=two)


def test_chunked_calls_mix_one_and_two_step_launches():
    case = layered_case(500, 40, nsteps=75)
    one = run_gpu(case, "f32", sum_rho=False, steps_per_launch=1)
    two = run_gpu(case, "f32", sum_rho=False, chunks=[1, 2, 3, 0, 5, 29, 35])
    same(one, two)


def test_sum_rho_recording_keeps_one_step_and_matches():
    """With the sum of rho recorded every step lb_step_n takes one step per
    launch; traces and fields equal those of the blocked path."""
    case = layered_case(400, 36, nsteps=50)
    a = run_gpu(case, "f32", sum_rho=True)
    b = run_gpu(case, "f32", sum_rho=False)
    same(a, b)


def test_two_step_vs_oracle_pulse_f64():
    """The 128^2 periodic Gaussian-pulse case (tau = 1, FP64) through the
    blocked path (four steps per launch): rho field against the oracle at
    the FP64 bar."""
    wl = inputs.pulse_workload()
    case = {"nx": 128, "ny": 128, "q": 5, "collision": "bgk", "tau": 1.0,
            "c2": wl["c2"], "rho0": wl["rho0"], "nsteps": wl["nsteps"],
            "receivers": np.array([(64, 64), (0, 0), (127, 127), (70, 64)], dtype=np.int32)}
    ref = run_oracle(case)
    compare(case, "f64", gpu=run_gpu(case, "f64", sum_rho=False), ref=ref)


def marching_receivers(nx, ny):
    """Receivers on the strip edges of the marching kernel (owned widths 112
    and 116 columns for seven and for five or six steps, 48, 50 and 56 for
    FP64's eight, seven and four), on its 20-row
    segment edges (and 24-row ones), on the periodic seam and in the
    sponge."""
    xs = {0, 1, nx - 1, nx - 2}
    for w in (112, 116, 48, 50, 56):
        for k in range(1, nx // w + 1):
            xs.update({k * w - 1, k * w, k * w + 1})
    ys = {0, 1, ny - 1, ny - 2}
    for h in (20, 24):
        for k in range(1, ny // h + 1):
            ys.update({h * k - 1, h * k, h * k + 1})
    xs = sorted(x for x in xs if 0 <= x < nx)
    ys = sorted(y for y in ys if 0 <= y < ny)
    return np.array([(x, y) for y in ys for x in xs[::2]] + [(x, ys[len(ys) // 2]) for x in xs],
                    dtype=np.int32)


@pytest.mark.parametrize("q,collision,s", [(5, "bgk", None), (5, "bgk", 0.8), (5, "mrt", [1, 1, 1, 1.6, 1.3]),
                                           (5, "mrt", [1, 1, 1, 2, 2]), (9, "bgk", None), (9, "bgk", 0.8),
                                           (9, "mrt", [1, 1, 1, 2, 2, 2, 1, 1, 2])])
@pytest.mark.parametrize("nx,ny", [(500, 40), (462, 36), (500, 34), (462, 33), (500, 32), (462, 31), (500, 30),
                                   (462, 29), (230, 41), (346, 71), (226, 97), (448, 48), (114, 64), (344, 61)])
def test_marching_kernel_shapes(q, collision, s, nx, ny):
    """FP32 grids that take the marching kernel (20-row segments; seven steps
    per launch for D2Q5 when ny >= 34, six for D2Q9 BGK when ny >= 32, five
    for D2Q9 MRT when ny >= 30) and
    grids just too short for it: heights around the thresholds, ragged last
    segments, widths that leave a partial last strip, step counts of every
    remainder, receivers and the source on strip and segment edges; bitwise
    equal to one step per launch and within the FP32 bar of the oracle."""
    tau = s if isinstance(s, float) else 0.5
    coll_s = None if isinstance(s, float) else s
    for nsteps, src in ((45, (min(112, nx - 1), 20)), (17, (min(116, nx - 1), 23)), (13, (nx - 1, ny - 1))):
        case = layered_case(nx, ny, q=q, collision=collision, tau=tau, s=coll_s, nsteps=nsteps, sponge=3)
        case["source"] = src
        case["wavelet"] = 1e2 * case["wavelet"]
        case["receivers"] = np.concatenate([case["receivers"], marching_receivers(nx, ny),
                                            np.array([src], dtype=np.int32)])
        two = both(case, "f32", spl=8)   # the marching kernel on grids of any size
        if nsteps == 45:
            compare(case, "f32", gpu=two)


@pytest.mark.parametrize("q,collision,s", [(5, "bgk", None), (5, "bgk", 0.8), (5, "mrt", [1, 1, 1, 1.6, 1.3]),
                                           (9, "bgk", None), (9, "mrt", [1, 1, 1, 2, 2, 2, 1, 1, 2])])
@pytest.mark.parametrize("nx,ny", [(301, 36), (300, 35), (250, 34), (251, 33), (200, 28), (199, 27), (147, 61),
                                   (96, 52)])
def test_marching_kernel_shapes_f64(q, collision, s, nx, ny):
    """FP64 grids that take the marching kernel (one column per lane,
    20-row segments; eight steps per launch for D2Q5 BGK when ny >= 36,
    seven for D2Q5 MRT when ny >= 34, four for D2Q9 when ny >= 28; odd
    widths included) and grids just too short for it: bitwise equal to one
    step per launch and within the FP64 bar of the oracle."""
    tau = s if isinstance(s, float) else 0.5
    coll_s = None if isinstance(s, float) else s
    for nsteps, src in ((41, (min(48, nx - 1), 20)), (11, (nx - 1, ny - 1))):
        case = layered_case(nx, ny, q=q, collision=collision, tau=tau, s=coll_s, nsteps=nsteps, sponge=3)
        case["source"] = src
        case["wavelet"] = 1e2 * case["wavelet"]
        case["receivers"] = np.concatenate([case["receivers"], marching_receivers(nx, ny),
                                            np.array([src], dtype=np.int32)])
        two = both(case, "f64", spl=8)
        if nsteps == 41:
            compare(case, "f64", gpu=two)


@pytest.mark.parametrize("collision,s", [("bgk", None), ("bgk", 0.8), ("mrt", [1, 1, 1, 1.6, 1.3])])
@pytest.mark.parametrize("nx,ny", [(500, 30), (500, 29), (464, 31), (228, 41), (348, 71), (448, 48)])
def test_marching_kernel_shapes_f16(collision, s, nx, ny):
    """D2Q5 with FP16 storage through the marching kernel (five steps per
    launch when nx is a multiple of 4 and ny >= 30; two columns per lane,
    116 owned per strip; 20-row segments) and grids just too short for it:
    bitwise equal to one step per launch."""
    tau = s if isinstance(s, float) else 0.5
    coll_s = None if isinstance(s, float) else s
    for nsteps, src in ((33, (min(116, nx - 1), 20)), (12, (nx - 1, ny - 1))):
        case = layered_case(nx, ny, q=5, collision=collision, tau=tau, s=coll_s, nsteps=nsteps, sponge=3)
        case["source"] = src
        case["wavelet"] = 1e2 * case["wavelet"]
        case["receivers"] = np.concatenate([case["receivers"], marching_receivers(nx, ny),
                                            np.array([src], dtype=np.int32)])
        both(case, "f16s", spl=8)
