"""The allocation-free h psi entry point (sky_apply_h_noalloc) against
sky_apply_h: same h psi and <psi|h psi>, bit for bit (the same kernels; the
partial sums only live in the library's fixed scratch instead of the
workspace), on two calls in a row, the second with fewer states; a request
beyond the fixed scratch is refused."""
import ctypes

import pytest

from paper_1610_07522_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_apply_h_matches(torch_mod, prec):
    torch = torch_mod
    from paper_1610_07522_amd import sky
    w = inputs.small_workload("na24", 24, 13, 7, init="rod", seed=60, noise=0.05)
    raw = inputs.raw_states(w)
    box = sky.Box(sky.desc_from_workload(w, precision=prec, twists=[(0.3, -0.7, 1.1)]))
    box.init_box(torch.from_numpy(raw[0]).cuda(), torch.from_numpy(raw[1]).cuda())
    for q, m in ((0, 13), (1, 5)):          # second call: fewer states
        psi = box.view("psi", q)
        h1, h2 = torch.empty_like(psi), torch.empty_like(psi)
        e1 = torch.zeros(psi.shape[0], dtype=torch.float64, device="cuda:0")
        e2 = torch.full_like(e1, float("nan"))
        box.apply_h(q, psi, h1, m, e1)
        box.apply_h_noalloc(q, psi, h2, m, e2)
        box.sync()
        assert torch.equal(h1[:m], h2[:m]), (prec, q)
        assert torch.equal(e1[:m], e2[:m]), (prec, q)
        assert torch.isnan(e2[m:]).all()


def test_noalloc_refuses_more_than_its_scratch():
    from paper_1610_07522_amd import sky
    lib = sky.load()
    w = inputs.small_workload("big", 64, 4200, 0, noise=0.0)
    d = sky.desc_from_workload(w)
    nb = ctypes.c_size_t()
    assert lib.sky_workspace_size(ctypes.byref(d), ctypes.byref(nb)) == sky.SKY_OK
    ctx = ctypes.c_void_p()
    fake = 1 << 40   # never dereferenced: the size check comes first
    assert lib.sky_create(ctypes.byref(d), fake, nb.value, None, ctypes.byref(ctx)) == sky.SKY_OK
    assert lib.sky_apply_h_noalloc(ctx, 0, fake, fake, 4200, fake) == sky.SKY_ERR_INVALID
    assert b"fixed scratch" in lib.sky_last_error()
    lib.sky_destroy(ctx)
