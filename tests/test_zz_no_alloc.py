"""The allocation-free selection entry point (vrm_select_diffused_static) against
vrm_select_diffused (Sec. 3.5) through the C ABI: bit-identical masks on two
calls in a row, the second with a smaller cloud (the fixed device state keeps
the first call's contents and must be cleared by the call), and the non-finite
flag."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vrm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_06379_amd as v
    v.lib()
    return v


def _context_mask(vrm, wl):
    cloud = vrm.Cloud(wl.x, wl.y, wl.gamma, capacity=wl.n + 64)
    ctx = vrm.Context(cloud.capacity)
    mask = torch.zeros(cloud.capacity, dtype=torch.uint8, device="cuda")
    ctx.vrm_select_diffused(cloud, vrm.params_of(wl), mask)
    torch.cuda.synchronize()
    return mask[:wl.n].cpu().numpy()


def test_static_selection_matches_the_context_entry_point(vrm):
    big = workloads.config_jittered(h=0.01, q=3, seed=2)            # 40 401 particles
    small = workloads.config_lattice_small()                          # 1 681 particles, q = 2
    flag = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    for wl in (big, small):
        ref = _context_mask(vrm, wl)
        g = torch.as_tensor(wl.gamma, device="cuda")
        mask = torch.full((wl.n + 64,), 7, dtype=torch.uint8, device="cuda")
        vrm.vrm_select_diffused_static(g, wl.n, wl.h, wl.q, wl.c_diff, mask, flag)
        torch.cuda.synchronize()
        got = mask[:wl.n].cpu().numpy()
        print(wl.name, "N", wl.n, "diffused", int(got.sum()), "context", int(ref.sum()), flush=True)
        np.testing.assert_array_equal(got, ref)
        assert int(flag.item()) == 0
        assert (mask[wl.n:].cpu().numpy() == 7).all()   # nothing past n written


def test_static_selection_flags_non_finite_and_rejects_bad_sizes(vrm):
    wl = workloads.config_lattice_small()
    g = torch.as_tensor(wl.gamma, device="cuda").clone()
    g[5] = float("nan")
    mask = torch.zeros(wl.n, dtype=torch.uint8, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    vrm.vrm_select_diffused_static(g, wl.n, wl.h, wl.q, wl.c_diff, mask, flag)
    torch.cuda.synchronize()
    assert int(flag.item()) == 2
    with pytest.raises(vrm.VrmError) as e:
        vrm.vrm_select_diffused_static(g, (1 << 26) + 1, wl.h, wl.q, wl.c_diff, mask, flag)
    assert e.value.code == vrm.E_ARG
