"""HIP-graph replay and batched uneven boxes, through the C ABI.

Graph replay is checked against the eager launches of the same context
after every iteration (several replays with host work between them), also
across the precision-ladder switch and on the learned step; the batched
driver is checked box by box against each box iterated alone, and one FP64
box of the batch against the oracle's trajectory.  Bar: the eager result
to 1e-12 relative (the same kernels on the same inputs; only the order of
floating-point atomics may differ), the oracle to 1e-10 relative.
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


def _box(w, precision=0, ladder_tol=0.0, stream=None):
    from paper_1610_07522_amd import sky
    return sky.Box(sky.desc_from_workload(w, precision=precision, ladder_tol=ladder_tol),
                   stream=stream)


def _init(box, w):
    raw = inputs.raw_states(w)
    box.init_box(to_dev(raw[0]), to_dev(raw[1]))


def _state(box):
    return [to_host(box.view("psi", q)).astype(np.complex128) for q in range(2)]


def _close(a, b, tol=1e-12):
    for x, y in zip(a, b):
        if x.size:
            assert np.abs(x - y).max() <= tol * max(np.abs(y).max(), 1e-300)


@pytest.mark.parametrize("case,precision,ladder", [("n24_13p7_rod", 0, 0.0),
                                                   ("n16_8p8", 1, 0.0),
                                                   ("n16_8p8", 1, 1e3)])
def test_graph_replay_matches_eager(torch_mod, case, precision, ladder):
    torch = torch_mod
    w = CASES[case]
    eager = _box(w, precision, ladder)
    graph = _box(w, precision, ladder, stream=torch.cuda.Stream())
    _init(eager, w)
    _init(graph, w)
    graph.set_graphs(True)
    for it in range(8):
        a = eager.iterate(1)
        b = graph.iterate(1)
        torch.cuda.synchronize()
        assert b["precision"] == a["precision"], it
        assert b["energy"] == pytest.approx(a["energy"], rel=1e-12, abs=0), it
        assert b["residual"] == pytest.approx(a["residual"], rel=1e-10, abs=0), it
        _close(_state(graph), _state(eager))
    if ladder > 0:   # switched after the first iteration: graphs recaptured in FP64
        assert a["precision"] == 0


def test_graph_replay_learned_step(torch_mod):
    torch = torch_mod
    w = CASES["n24_13p7_rod"]
    boxes = [_box(w), _box(w, stream=torch.cuda.Stream())]
    for b in boxes:
        _init(b, w)
        b.iterate(3)
        b.precond_collect(0)
        b.precond_collect(1)
        b.precond_train(20, 1e-3)
        b.precond_use(True, -1.0, 0)
    boxes[1].set_graphs(True)
    for it in range(4):
        r = [b.iterate(1) for b in boxes]
        torch.cuda.synchronize()
        assert r[0]["precond_iters"] == r[1]["precond_iters"] == 1
        assert r[1]["energy"] == pytest.approx(r[0]["energy"], rel=1e-11, abs=0), it
        _close(_state(boxes[1]), _state(boxes[0]), 1e-10)


BATCH = [
    ("n16_8p8", 0),
    ("n24_13p7_rod", 1),
    ("n8_5p3", 0),
    ("n32_70p33_slab", 1),
    ("n24_13p7_rod", 0),
    ("n16_8p8", 1),
]


@pytest.mark.parametrize("nthreads", [1, 3, 8])
def test_batch_matches_boxes_alone(torch_mod, nthreads):
    from paper_1610_07522_amd import sky
    torch = torch_mod
    K = 4
    batch, alone = [], []
    for case, prec in BATCH:
        w = CASES[case]
        b = _box(w, prec)
        _init(b, w)
        batch.append(b)
        a = _box(w, prec)
        _init(a, w)
        alone.append(a)
    reps = sky.batch_iterate(batch, nthreads, K)
    torch.cuda.synchronize()
    for (case, prec), b, a, r in zip(BATCH, batch, alone, reps):
        ra = a.iterate(K)
        assert r["iters"] == K
        assert r["energy"] == pytest.approx(ra["energy"], rel=1e-12, abs=0), case
        _close(_state(b), _state(a))
    # one FP64 box of the batch against the oracle trajectory
    w = CASES["n16_8p8"]
    raw = inputs.raw_states(w)
    st = so.initial_state(raw[0], raw[1], Grid(w.n, w.dx), w.params, w.damp_x0, w.damp_e0)
    for _ in range(K):
        rep = so.iterate(st)
    assert reps[0]["energy"] == pytest.approx(rep.E["total"], rel=1e-10, abs=0)


def test_batch_per_box_tolerance(torch_mod):
    from paper_1610_07522_amd import sky
    torch = torch_mod
    cases = [("n16_8p8", 0), ("n8_5p3", 0), ("n24_13p7_rod", 1)]
    tol = 0.1
    batch, alone = [], []
    for case, prec in cases:
        w = CASES[case]
        for lst in (batch, alone):
            b = _box(w, prec)
            _init(b, w)
            lst.append(b)
    reps = sky.batch_iterate(batch, 2, 1000, tol)
    torch.cuda.synchronize()
    iters = []
    for (case, _), a, r in zip(cases, alone, reps):
        ra = a.iterate(1000, tol)
        assert r["converged"] and r["residual"] <= tol, case
        assert r["iters"] == ra["iters"], case
        assert r["energy"] == pytest.approx(ra["energy"], rel=1e-11, abs=0), case
        iters.append(r["iters"])
    assert len(set(iters)) > 1   # boxes stopped at their own iteration counts
