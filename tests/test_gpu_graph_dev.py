"""The device-decided iteration (sky_iterate_graph, sky_batch_iterate_graph)
through the C ABI.

Every decision of an iteration -- the Loewdin series' term count, the
refinement's stop test, Delta-eps and the stop at the tolerance -- is taken
on the device and the whole iteration is replayed as one HIP graph; the host
reads a box's flags once per chunk.  Checked against sky_iterate on the same
boxes: the same kernels on the same inputs in the same order (only Delta-eps
is summed in another order, and it feeds nothing back), so states and
energies to 1e-12 relative in both precisions; iteration counts at a
tolerance equal.  The hand-over to the host (a refinement that does not
converge within the device's step budget) is forced with a one-step budget
and must give sky_iterate's trajectory.  One FP64 box against the oracle.
"""
import numpy as np
import pytest

from oracle import Grid
from oracle import solver as so
from paper_1610_07522_amd import inputs

from gpu_util import CASES, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _box(w, precision=0, ladder_tol=0.0, stream=None, dev_refine_steps=0):
    from paper_1610_07522_amd import sky
    d = sky.desc_from_workload(w, precision=precision, ladder_tol=ladder_tol)
    d.dev_refine_steps = dev_refine_steps
    return sky.Box(d, stream=stream)


def _init(box, w):
    raw = inputs.raw_states(w)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))


def _state(box):
    return [to_host(box.view("psi", q)).astype(np.complex128) for q in range(2)]


def _close(a, b, tol):
    for x, y in zip(a, b):
        if x.size:
            assert np.abs(x - y).max() <= tol * max(np.abs(y).max(), 1e-300)


@pytest.mark.parametrize("case,precision,chunk", [("n24_13p7_rod", 0, 3), ("n16_8p8", 1, 4),
                                                  ("n32_70p33_slab", 0, 16)])
def test_iterate_graph_matches_host_path(torch_mod, case, precision, chunk):
    torch = torch_mod
    w = CASES[case]
    host = _box(w, precision)
    dev = _box(w, precision, stream=torch.cuda.Stream())
    _init(host, w)
    _init(dev, w)
    K = 7
    ra = host.iterate(K)
    rb = dev.iterate_graph(K, 0.0, chunk)
    torch.cuda.synchronize()
    assert rb["iters"] == K
    tol_e = tol_s = 1e-12
    assert rb["energy"] == pytest.approx(ra["energy"], rel=tol_e, abs=0)
    assert rb["residual"] == pytest.approx(ra["residual"], rel=1e-9, abs=0)
    _close(_state(dev), _state(host), tol_s)
    # a second call continues from there
    ra = host.iterate(2)
    rb = dev.iterate_graph(2, 0.0, chunk)
    assert rb["energy"] == pytest.approx(ra["energy"], rel=tol_e, abs=0)
    assert dev.iteration() == host.iteration() == K + 2


def test_iterate_graph_handover_to_host(torch_mod):
    """A one-step refinement budget: sets whose refinement needs more steps
    are handed to the host path mid-iteration and finished there."""
    torch = torch_mod
    w = CASES["n24_13p7_rod"]
    host = _box(w)
    dev = _box(w, stream=torch.cuda.Stream(), dev_refine_steps=1)
    _init(host, w)
    _init(dev, w)
    K = 6
    ra = host.iterate(K)
    rb = dev.iterate_graph(K, 0.0, 2)
    torch.cuda.synchronize()
    assert rb["iters"] == K
    assert rb["eig_fallbacks"] > 0          # hand-overs happened
    assert rb["energy"] == pytest.approx(ra["energy"], rel=1e-12, abs=0)
    _close(_state(dev), _state(host), 1e-12)


def test_iterate_graph_tolerance_and_oracle(torch_mod):
    """Stop at Delta-eps <= tol on the device: the same iteration count as
    sky_iterate; the FP64 box's energy against the oracle's trajectory."""
    torch = torch_mod
    w = CASES["n16_8p8"]
    tol = 0.1
    host = _box(w)
    dev = _box(w, stream=torch.cuda.Stream())
    _init(host, w)
    _init(dev, w)
    ra = host.iterate(500, tol)
    rb = dev.iterate_graph(500, tol, 8)
    torch.cuda.synchronize()
    assert ra["converged"] and rb["converged"]
    assert rb["iters"] == ra["iters"]
    assert rb["residual"] <= tol
    assert rb["energy"] == pytest.approx(ra["energy"], rel=1e-12, abs=0)
    raw = inputs.raw_states(w)
    st = so.initial_state(raw[0], raw[1], Grid(w.n, w.dx), w.params, w.damp_x0, w.damp_e0)
    for _ in range(rb["iters"]):
        rep = so.iterate(st)
    assert rb["energy"] == pytest.approx(rep.E["total"], rel=1e-10, abs=0)


BATCH = [
    ("n16_8p8", 0, 0.0),
    ("n24_13p7_rod", 1, 0.0),
    ("n8_5p3", 0, 0.0),
    ("n32_70p33_slab", 1, 0.0),
    ("n24_13p7_rod", 0, 0.0),
    ("n16_8p8", 1, 1e3),     # ladder: host-decided, runs the host path inside the batch
]


@pytest.mark.parametrize("nthreads,tol", [(1, 0.0), (3, 0.0), (4, 0.1)])
def test_batch_graph_matches_boxes_alone(torch_mod, nthreads, tol):
    from paper_1610_07522_amd import sky
    torch = torch_mod
    K = 5 if tol == 0.0 else 400
    batch, alone = [], []
    for case, prec, ladder in BATCH:
        w = CASES[case]
        for lst in (batch, alone):
            b = _box(w, prec, ladder)
            _init(b, w)
            lst.append(b)
    reps = sky.batch_iterate_graph(batch, nthreads, K, tol, 4)
    torch.cuda.synchronize()
    iters = []
    conv = []
    for (case, prec, ladder), b, a, r in zip(BATCH, batch, alone, reps):
        ra = a.iterate(K, tol)
        assert r["iters"] == ra["iters"], case
        assert r["converged"] == ra["converged"], case
        if tol > 0 and r["converged"]:
            assert r["residual"] <= tol
            conv.append(r["iters"])
        assert r["energy"] == pytest.approx(ra["energy"], rel=1e-12, abs=0), case
        _close(_state(b), _state(a), 1e-12)
        iters.append(r["iters"])
    if tol > 0:
        assert len(set(conv)) > 1   # converged boxes stopped at their own iterations


def test_iterate_graph_nan_reports_nan(torch_mod):
    """A NaN in one state: the device hands the set over (the overlap norm is
    not finite) and the host path reports SKY_ERR_NAN."""
    from paper_1610_07522_amd import sky
    torch = torch_mod
    w = inputs.small_workload("nan8", 8, 5, 3, init="slab", seed=51, noise=0.2)
    raw = inputs.raw_states(w)
    box = _box(w, stream=torch.cuda.Stream())
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))
    bad = raw[0].copy()
    bad[2, 0, 3, 4, 5] = np.nan
    box.set_states(0, to_dev(bad))
    with pytest.raises(sky.SkyError) as e:
        box.iterate_graph(3, 0.0, 2)
    assert e.value.code == sky.SKY_ERR_NAN
