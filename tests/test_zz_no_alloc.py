"""The entry point that allocates nothing (clusco_crmsd_matrix_noalloc),
called through the C ABI, against the entry point with a caller workspace
(clusco_crmsd_matrix) on the same inputs, and against the FP64 oracle.

Both entry points run the same kernels, so their scores must be identical
bit for bit; the oracle check uses the precision's tolerance.  Two calls in
a row, the second smaller, show that what the built-in scratch keeps from
the first call does not leak into the second; the oversize case shows the
host-side refusal."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1302_4000_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16": 5e-4, "fp16": 1e-4, "fp64": 1e-6, "bf16x4": 5e-4}


@pytest.fixture(scope="module")
def cl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_4000_amd as m
    for p, t in TOL.items():
        m.set_tolerance(p, t)
    return m


def say(*a):
    print(*a, flush=True)


def noalloc(cl, xd, prec):
    """Direct ctypes call of the C entry point, into a preallocated output."""
    b = cl.binding
    N, L = xd.shape[0], xd.shape[1]
    out = torch.full((N * (N - 1) // 2,), -1.0, dtype=torch.float32, device=xd.device)
    torch.cuda.synchronize()
    h = b.handle(xd.device.index)
    rc = b.lib().clusco_crmsd_matrix_noalloc(h, ctypes.c_void_p(xd.data_ptr()), N, L,
                                             b.PRECISION[prec], ctypes.c_void_p(out.data_ptr()),
                                             b._stream(xd.device))
    assert rc == b.OK, b.lib().clusco_last_error(h)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "fp64", "bf16x4"])
def test_noalloc_matches_workspace_entry(cl, prec):
    # large then small: stale scratch contents from the first call must not
    # reach the second (fix-up list, counters, operands of other models)
    for seed, N, L in ((31, 700, 150), (32, 97, 61)):
        say(f"[no-alloc] {prec} N={N} L={L} seed={seed}")
        x = synth.make_ensemble(seed, N, L, sigma=(0.2, 4.0), near_identical=20)
        xd = torch.from_numpy(x).cuda()
        got = noalloc(cl, xd, prec)
        ref = cl.crmsd_matrix(xd, prec)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(g.view(np.uint32), r.view(np.uint32)), \
            f"{prec} N={N}: {int((g != r).sum())} scores differ"
        err = float(np.abs(g.astype(np.float64) - oracle.crmsd_matrix(x)).max())
        say(f"  bit-equal to clusco_crmsd_matrix; max err vs oracle {err:.3e} A")
        assert err < TOL[prec]


def test_noalloc_rejects_oversize(cl):
    b = cl.binding
    h = b.handle(0)
    N, L = 60000, 150
    need = b.lib().clusco_crmsd_workspace_size(h, N, L, b.PRECISION["bf16"])
    assert need > b.SCRATCH_BYTES
    say(f"[no-alloc] oversize N={N} L={L}: workspace {need} > {b.SCRATCH_BYTES}")
    x = torch.zeros(1, dtype=torch.float32, device="cuda")
    o = torch.zeros(1, dtype=torch.float32, device="cuda")
    rc = b.lib().clusco_crmsd_matrix_noalloc(h, ctypes.c_void_p(x.data_ptr()), N, L,
                                             b.PRECISION["bf16"], ctypes.c_void_p(o.data_ptr()),
                                             b._stream(x.device))
    assert rc == b.ERR_UNSUPPORTED
    assert b"scratch" in b.lib().clusco_last_error(h)
    torch.cuda.synchronize()
