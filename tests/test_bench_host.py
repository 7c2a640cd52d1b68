"""Host-side checks of bench.py's roofline and HBM-phase arithmetic (CPU).

Fed the phase times of a plausible 48^3 x 1600 mixed iteration, the derived
figures must respect what the hardware and the method allow: no rate above
its peak, the method's flops at most a third of the FP16 peak (three split
products per real product), counted HBM bytes never below the compulsory
bytes of the phase, and the compulsory bytes of a phase a whole number of
state arrays.  A corrupted constant (a count overwritten, a peak in the wrong
unit) fails one of these.
"""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _timing(ms):
    return {k: dict(ms_n=2 * v, ms_p=0.5 * v, launches_n=2, launches_p=2) for k, v in ms.items()}


PHASE_MS = dict(apply_h=4.9, damp=5.8, densities=2.8, overlap_gemm=12.7, combine_gemm=11.0,
                subspace=5.8, meanfield=0.4, split=1.8)


def test_hbm_phases_respect_peaks_and_compulsory_bytes(bench):
    from paper_1610_07522_amd import inputs
    w = inputs.WORKLOADS["rod48"]
    out = bench.hbm_phases(_timing(PHASE_MS), w, True)
    state_bytes = 2 * w.n ** 3 * w.n_neutrons * 8
    for ph in ("apply_h", "damp", "densities"):
        r = out[ph]
        assert isinstance(r["state_arrays"], int) and 1 <= r["state_arrays"] <= 3, ph
        assert r["bytes_per_launch"] == r["state_arrays"] * state_bytes, ph
        assert 0.0 < r["frac"] < 1.0, ph
        if "counter_bytes" in r:
            assert r["counter_bytes"] >= r["bytes_per_launch"], ph
            assert 0.0 < r["counter_frac"] < 1.0, ph


def test_roofline_respects_split_bound_and_traffic(bench):
    from paper_1610_07522_amd import inputs
    w = inputs.WORKLOADS["rod48"]
    r = bench.roofline(_timing(PHASE_MS), w, True)
    assert r["kernel"] == "k_overlap_planes"
    assert 0.0 < r["frac"] <= 1.0 / bench.SPLIT_PRODUCTS
    assert 0.0 < r["issued"]["frac"] <= 1.0
    assert r["per_launch"]["flops"] == 8.0 * 2 * (1600 * 1601 // 2) * 2 * 48 ** 3
    if r["traffic"] is not None:
        assert r["traffic"] >= r["per_launch"]["unique_bytes"]
    r64 = bench.roofline(_timing(dict(PHASE_MS, overlap_gemm=80.0, combine_gemm=75.0)), w, False)
    assert r64["kernel"] == "k_overlap_lower" and 0.0 < r64["frac"] <= 1.0
