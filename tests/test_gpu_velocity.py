"""Biot-Savart velocity of the particles (Sec. 3.4 eq. nsode, with the
regularised kernel K_eps of Sec. 5) on the GPU, through the C ABI, against the
FP64 oracle: whole clouds up to 10^4 particles, sampled targets of the
40k-particle cloud, edge cases; plus the kernel's rate (16 FLOP per pair:
two differences, |d|^2, the exponent's scale, exp, 1 - e, reciprocal, two
products and two accumulations) against the FP32 VALU peak without packed math.
FP32 with the hardware exp2 and reciprocal: velocities within 1e-5 relative L2."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FLOP_PER_PAIR = 16
PEAK_TFLOPS = 78.6


@pytest.fixture(scope="module")
def vrm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_06379_amd as v
    v.lib()
    return v


def _say(*a):
    print(*a, flush=True)


def _clouds():
    h = 0.02
    x, y = workloads.lattice(-1.0, 1.0, h)
    lam = (x.astype(np.float32), y.astype(np.float32),
           (workloads.lamb_oseen_omega(x, y, 1.0, 0.01, 1.0) * h * h).astype(np.float32), 3 * h)
    wl = workloads.config_jittered(h=0.02, q=2, seed=2)
    jit = (wl.x, wl.y, wl.gamma, 3 * 0.02)
    rng = np.random.default_rng(11)
    n = 5003
    rnd = (rng.uniform(-1, 1, n).astype(np.float32), rng.uniform(-1, 1, n).astype(np.float32),
           rng.normal(0, 1, n).astype(np.float32), 0.05)
    return {"lamb_oseen_lattice_h0.02": lam, "jittered_h0.02": jit, "random_signed_5003": rnd}


CLOUDS = _clouds()


def _gpu_velocity(vrm, x, y, g, eps):
    cloud = vrm.Cloud(x, y, g, capacity=x.size + 64)
    ctx = vrm.Context(cloud.capacity)
    u = torch.full((cloud.capacity,), 7.0, device="cuda")
    v = torch.full((cloud.capacity,), 7.0, device="cuda")
    ctx.vrm_biot_savart(cloud, eps, u, v)
    torch.cuda.synchronize()
    return u[:x.size].cpu().numpy().astype(np.float64), v[:x.size].cpu().numpy().astype(np.float64), (ctx, cloud, u, v)


def _rel(a, b):
    return np.linalg.norm(np.concatenate(a) - np.concatenate(b)) / np.linalg.norm(np.concatenate(b))


@pytest.mark.parametrize("name", list(CLOUDS))
def test_biot_savart_matches_oracle(vrm, orc, name):
    x, y, g, eps = CLOUDS[name]
    _say("case", name, x.size)
    u, v, _ = _gpu_velocity(vrm, x, y, g, eps)
    ru, rv = orc.biot_savart(x, y, g, eps)
    err = _rel((u, v), (ru, rv))
    _say(name, "rel L2", err)
    assert err <= 1e-5


def test_biot_savart_edges(vrm, orc):
    # one particle: no velocity; two: equal and opposite momentum
    u, v, _ = _gpu_velocity(vrm, np.array([0.25], np.float32), np.array([-0.5], np.float32),
                            np.array([3.0], np.float32), 0.1)
    assert u[0] == 0.0 and v[0] == 0.0
    x = np.array([0.0, 0.1], np.float32)
    y = np.array([0.0, 0.05], np.float32)
    g = np.array([1.0, -2.0], np.float32)
    u, v, _ = _gpu_velocity(vrm, x, y, g, 0.07)
    ru, rv = orc.biot_savart(x, y, g, 0.07)
    assert _rel((u, v), (ru, rv)) <= 1e-6
    with pytest.raises(vrm.VrmError):
        _gpu_velocity(vrm, x, y, g, 0.0)


@pytest.mark.timeout(300)
def test_biot_savart_full_size_sampled_and_rate(vrm, orc):
    """The 40k-particle cloud (h = 0.01, eps = 3h): 600 sampled targets against the
    oracle's sums over all sources; then the kernel's rate."""
    wl = workloads.config_jittered(h=0.01, q=2, seed=2)
    eps = 0.03
    u, v, (ctx, cloud, ud, vd) = _gpu_velocity(vrm, wl.x, wl.y, wl.gamma, eps)
    sel = np.random.default_rng(3).choice(wl.n, 600, replace=False)
    ru, rv = orc.biot_savart(wl.x, wl.y, wl.gamma, eps, wl.x[sel], wl.y[sel])
    err = _rel((u[sel], v[sel]), (ru, rv))
    _say("sampled rel L2", err)
    assert err <= 1e-5
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    a.record()
    for _ in range(reps):
        ctx.vrm_biot_savart(cloud, eps, ud, vd)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    pairs = float(wl.n) ** 2
    tflops = pairs * FLOP_PER_PAIR / (ms * 1e-3) / 1e12
    _say(f"N {wl.n}: {ms:.3f} ms per evaluation, {pairs / ms / 1e6:.1f} G pairs/s, {tflops:.1f} TFLOP/s "
         f"= {tflops / PEAK_TFLOPS:.3f} of {PEAK_TFLOPS}")
