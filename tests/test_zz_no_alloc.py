"""The allocation-free expectation, pp_expectation_noalloc, through the C ABI.

Two calls in a row on one GPU, the second on a smaller observable, each against
pp_expectation on the same observable (FP64 bar: 1e-10 absolute; the two sum the diagonal
terms in different orders).  The first observable has more terms than 2048 workgroups of 256
threads cover in one sweep, so the workgroups stride.  Neither call may allocate device
memory: the context's allocator hook counts every allocation the library makes, and torch's
caching allocator counts every block it hands out.
"""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2606_20441_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _call_noalloc(pp, obs, basis=None):
    out = C.c_double(float("nan"))
    b = None
    if basis is not None:
        b = np.ascontiguousarray(np.asarray(basis, np.uint64).reshape(-1))
        b = b.ctypes.data_as(C.POINTER(C.c_uint64))
    rc = pp.lib().pp_expectation_noalloc(obs._h, b, C.byref(out))
    assert rc == 0, pp.lib().pp_last_error()
    return out.value


def test_expectation_noalloc_two_calls():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_20441_amd import pp
    ctx = pp.Context(0)
    big = W.random_pauli_arrays(56, 700_000, seed=41, density=0.3)
    big.x[: 300_000] = 0                       # a large diagonal share
    small = W.random_pauli_sum(56, 300, seed=42)
    small.x[:120] = 0
    rng = np.random.default_rng(43)
    basis = np.zeros(1, np.uint64)
    for q in rng.choice(56, 20, replace=False):
        basis[0] |= np.uint64(1) << np.uint64(int(q))
    for name, ps in (("700000 terms", big), ("300 terms", small)):
        log(f"no-alloc expectation: {name}")
        g = pp.Observable.from_sum(ctx, ps)
        for b in (None, basis):
            want = g.expectation(b)
            torch.cuda.synchronize()
            n0 = ctx.n_allocs
            s0 = torch.cuda.memory_stats(0).get("allocation.all.allocated", 0)
            got = _call_noalloc(pp, g, b)
            torch.cuda.synchronize()
            assert ctx.n_allocs == n0, "the library allocated device memory"
            assert torch.cuda.memory_stats(0).get("allocation.all.allocated", 0) == s0
            log(f"  basis {'|0>' if b is None else 'b'}: {got!r} vs pp_expectation {want!r}")
            assert abs(got - want) < 1e-10
        g.destroy()
    # argument errors are reported, not raised as device faults
    out = C.c_double()
    assert pp.lib().pp_expectation_noalloc(None, None, C.byref(out)) == pp.PP_ERR_INVALID
    ctx.close()
