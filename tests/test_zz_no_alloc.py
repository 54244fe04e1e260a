"""mm_modp_static (no allocation, fixed per-device workspace) against
mm_modp_async, through the C-ABI, tolerance 0.

Each case makes two calls in a row on one device, the second with a smaller
product, so the second reads a workspace the first has filled; both results
must equal mm_modp_async's and the oracle's.  Collected last: its workspace
is shared by every call on the device.
"""
import ctypes
import sys

import numpy as np
import pytest

import mmp_inputs as gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mmp = pytest.importorskip("paper_2601_07508_amd")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def call(entry, A, B, C, p, u=0, v=0, **opts):
    """One call of a C entry point (mm_modp_static or mm_modp_async) on torch's stream."""
    o = mmp._opts(**opts)
    m, k = A.shape
    n = B.shape[1]
    fn = getattr(mmp.lib(), entry)
    return fn(ctypes.byref(o), p, u, v, m, n, k, ctypes.c_void_p(A.data_ptr()), A.stride(0),
              ctypes.c_void_p(B.data_ptr()), B.stride(0), ctypes.c_void_p(C.data_ptr()), C.stride(0),
              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


# (p, u, v, options, large shape, smaller shape): the INT8 form (digit planes
# in the workspace), FP64 words with split-K (k-range residues in it), and
# the INT8 form with split-K (both)
CASES = [
    (1125899906842597, 0, 0, {"form": 2}, (700, 600, 900), (130, 70, 300)),
    (68719476731, 0, 0, {"form": 2, "splits": 4}, (96, 80, 20000), (33, 17, 5000)),
    (67108859, 1, 2, {"splits": 8}, (100, 100, 40000), (40, 9, 7000)),
    (4503599627370449, 0, 0, {}, (1024, 512, 768), (64, 64, 64)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_static_equals_async_twice(case):
    p, u, v, opts, big, small = CASES[case]
    for r, (m, n, k) in enumerate((big, small)):
        say("no-alloc case", case, "call", r, (m, n, k), p, opts)
        A = gen.random_matrix(case * 10 + r, 1, m, k, p)
        B = gen.random_matrix(case * 10 + r, 2, k, n, p)
        dA, dB = dev(A), dev(B)
        Cs = torch.full((m, n), -1.0, dtype=torch.float64, device="cuda")
        Ca = torch.full((m, n), -2.0, dtype=torch.float64, device="cuda")
        assert call("mm_modp_static", dA, dB, Cs, p, u, v, **opts) == 0
        assert call("mm_modp_async", dA, dB, Ca, p, u, v, **opts) == 0
        torch.cuda.synchronize()
        assert torch.equal(Cs, Ca)
        assert np.array_equal(Cs.cpu().numpy(), oracle.mm_modp(p, A, B).astype(np.float64))


def test_static_rejects_beyond_its_workspace():
    # 16384 x 16384 x 4096 in the INT8 form at 52 bits needs about 0.9 GB of
    # digit planes: refused on the host before any device work
    p = 4503599627370449
    m = n = 16384
    k = 4096
    pl = mmp.plan(p, m, n, k, form=2, splits=1)
    assert pl["workspace_bytes"] > mmp.STATIC_SCRATCH_BYTES
    A = torch.empty((m, k), dtype=torch.float64, device="cuda")
    B = torch.empty((k, n), dtype=torch.float64, device="cuda")
    C = torch.full((m, n), -1.0, dtype=torch.float64, device="cuda")
    assert call("mm_modp_static", A, B, C, p, form=2, splits=1) == -4  # MMP_ENOMEM
    torch.cuda.synchronize()
    assert bool(torch.all(C == -1.0))
    # a caller workspace or entry validation is refused too
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    small = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    assert call("mm_modp_static", small, small, small.clone(), p, workspace=ws) == -1
    assert call("mm_modp_static", small, small, small.clone(), p, validate_entries=True) == -1
