"""GPU checks of the vector-operation and transfer micro-benchmarks (the
MI355X counterparts of the paper's Tables 2 and 5): the arithmetic ops are
bit-exact against NumPy float32 (IEEE single, correctly rounded), sin, cos,
log and exp within 4 ulp of the double-precision value, and whole and
border-only transfers move exactly the sites they name."""
import numpy as np
import pytest

from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_cs_0312006_amd import binding
    binding.lib()
    return binding, torch


def _ulp_err(got, ref64):
    ref32 = ref64.astype(np.float32)
    spacing = np.spacing(np.abs(ref32)).astype(np.float64)
    return np.abs(got.astype(np.float64) - ref64) / spacing


@pytest.mark.parametrize("n", [4 * 256 * 256, 4 * 512 * 512, 1001, 4, 3])
@pytest.mark.parametrize("op", ["=", "+", "-", "*", "/", "sin", "cos", "log", "exp"])
def test_vector_op(env, op, n):
    b, torch = env
    rng = np.random.default_rng(n)
    if op == "log":
        a0 = rng.uniform(1e-3, 1e3, n).astype(np.float32)
    elif op == "exp":
        a0 = rng.uniform(-80, 80, n).astype(np.float32)
    elif op in ("sin", "cos"):
        a0 = rng.uniform(-100, 100, n).astype(np.float32)
    else:
        a0 = rng.standard_normal(n).astype(np.float32)
    c0 = rng.standard_normal(n).astype(np.float32) + np.float32(3.0)
    a = torch.from_numpy(a0).cuda()
    c = torch.from_numpy(c0).cuda()
    G.log(f"vector op {op} n={n}")
    b.mb_vector_op(op, a.data_ptr(), c.data_ptr(), n)
    torch.cuda.synchronize()
    got = a.cpu().numpy()
    exact = {"=": c0, "+": a0 + c0, "-": a0 - c0, "*": a0 * c0, "/": a0 / c0}
    if op in exact:
        assert np.array_equal(got.view(np.uint32), exact[op].view(np.uint32))
    else:
        ref = {"sin": np.sin, "cos": np.cos, "log": np.log, "exp": np.exp}[op](a0.astype(np.float64))
        assert _ulp_err(got, ref).max() <= 4.0


@pytest.mark.parametrize("L,elem", [(64, 1), (127, 16), (512, 4), (2, 4), (1, 1)])
def test_transfers_whole_and_border(env, L, elem):
    b, torch = env
    rng = np.random.default_rng(L)
    host = torch.from_numpy(rng.integers(0, 256, (L, L * elem), dtype=np.uint8)).pin_memory()
    dev = torch.zeros((L, L * elem), dtype=torch.uint8, device="cuda")
    G.log(f"transfer L={L} elem={elem}")
    b.mb_copy_lattice(dev.data_ptr(), host.data_ptr(), L, elem, b.MB_HOST_TO_DEVICE, border=True)
    torch.cuda.synchronize()
    d = dev.cpu().numpy().reshape(L, L, elem)
    h = host.numpy().reshape(L, L, elem)
    mask = np.zeros((L, L), dtype=bool)
    mask[0] = mask[-1] = True
    mask[:, 0] = mask[:, -1] = True
    assert np.array_equal(d[mask], h[mask]) and np.all(d[~mask] == 0)
    back = torch.zeros_like(host).pin_memory()
    b.mb_copy_lattice(back.data_ptr(), dev.data_ptr(), L, elem, b.MB_DEVICE_TO_HOST, border=True)
    torch.cuda.synchronize()
    assert np.array_equal(back.numpy().reshape(L, L, elem)[mask], h[mask])
    b.mb_copy_lattice(dev.data_ptr(), host.data_ptr(), L, elem, b.MB_HOST_TO_DEVICE, border=False)
    b.mb_copy_lattice(back.data_ptr(), dev.data_ptr(), L, elem, b.MB_DEVICE_TO_HOST, border=False)
    torch.cuda.synchronize()
    assert np.array_equal(back.numpy(), host.numpy())


def test_philox_rate_kernel_draws_philox(env):
    """The Philox-rate kernel evaluates the same draws as the NumPy Philox:
    each thread's XOR of the words of counters (thread, k, 0, 0)."""
    from oracle import mini
    b, torch = env
    n, calls, seed = 1000, 5, 0x1234567890ABCDEF
    out = torch.zeros(n, dtype=torch.int32, device="cuda")
    G.log("philox rate kernel n=1000 calls=5")
    b.mb_philox(out.data_ptr(), n, calls, seed)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    tid = np.arange(n, dtype=np.uint64)
    acc = np.zeros(n, dtype=np.uint64)
    for k in range(calls):
        w = mini.philox4x32_10(tid, k, 0, 0, seed & 0xFFFFFFFF, seed >> 32)
        acc ^= w[0] ^ w[1] ^ w[2] ^ w[3]
    assert np.array_equal(got, acc.astype(np.uint32))
