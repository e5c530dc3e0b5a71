"""sft_execute_noalloc (the entry point for callers that cannot allocate device
memory) against sft_execute: the same kernels, so the outputs must be bitwise
equal; two calls in a row through the C ABI, the second with a smaller input,
so the second runs over the first's leftover scratch contents.  The plans used
here never run anything but the no-alloc call before it is checked, so their
own workspace must stay unallocated."""
import ctypes

import numpy as np
import pytest
import torch

import siggen

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _outputs(s, dev, fill):
    return (torch.full((s,), fill, dtype=torch.int64, device=dev),
            torch.full((s,), complex(fill, -fill), dtype=torch.complex64, device=dev),
            torch.full((1,), fill, dtype=torch.int32, device=dev))


def _run(lib, fn, plan, f, out, stream):
    rc = fn(plan.handle, _vp(f), _vp(out[0]), _vp(out[1]), _vp(out[2]), ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0, lib.sft_last_error().decode()


def test_noalloc_equals_execute_twice_second_smaller(gpu):
    lib = gpu.load_library()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sigs = [siggen.workload("plain_n2e22_s64_20db", 3),
            siggen.sparse_signal(2 ** 16, 16, 5, 20.0)]
    assert sigs[1].N < sigs[0].N
    for sig in sigs:
        print(f"[no-alloc] N={sig.N} s={sig.s}", flush=True)
        ref_plan = gpu.Plan(sig.N, sig.s)
        na_plan = gpu.Plan(sig.N, sig.s)
        assert na_plan.workspace_bytes() <= SCRATCH_BYTES
        fp0 = na_plan.footprint()
        f = torch.from_numpy(sig.f32).to(dev)
        ref = _outputs(sig.s, dev, 7)
        got = _outputs(sig.s, dev, -3)
        _run(lib, lib.sft_execute, ref_plan, f, ref, stream)
        _run(lib, lib.sft_execute_noalloc, na_plan, f, got, stream)
        torch.cuda.synchronize()
        assert na_plan.status() == 0
        # the no-alloc call must not have created the plan's own workspace
        assert na_plan.footprint() == fp0
        n_ref, n_got = int(ref[2].item()), int(got[2].item())
        assert n_ref == n_got and n_ref > 0
        assert torch.equal(ref[0], got[0])
        assert torch.equal(torch.view_as_real(ref[1]), torch.view_as_real(got[1]))
        # also against the known support of the input (unit coefficients, 20 dB)
        assert sorted(got[0][:n_got].cpu().tolist()) == sorted(int(w) for w in sig.freqs)


def test_noalloc_allocates_nothing_on_repeat(gpu):
    lib = gpu.load_library()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sig = siggen.sparse_signal(2 ** 18, 32, 11, 30.0)
    plan = gpu.Plan(sig.N, sig.s)
    f = torch.from_numpy(sig.f32).to(dev)
    out = _outputs(sig.s, dev, 0)
    _run(lib, lib.sft_execute_noalloc, plan, f, out, stream)   # first call on the device: symbol lookup
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info(dev)
    for _ in range(5):
        _run(lib, lib.sft_execute_noalloc, plan, f, out, stream)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info(dev)
    assert free1 == free0
    assert plan.status() == 0


def test_noalloc_rejects_a_workspace_beyond_the_scratch(gpu):
    lib = gpu.load_library()
    dev = torch.device("cuda:0")
    N, s = 2 ** 26, 1024
    plan = gpu.Plan(N, s)
    assert plan.workspace_bytes() > SCRATCH_BYTES
    f = torch.zeros(N, dtype=torch.complex64, device=dev)
    out = _outputs(s, dev, 9)
    rc = lib.sft_execute_noalloc(plan.handle, _vp(f), _vp(out[0]), _vp(out[1]), _vp(out[2]),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == gpu.SFT_EINVAL
    assert "scratch" in lib.sft_last_error().decode()
    torch.cuda.synchronize()
    assert int(out[2].item()) == 9   # nothing was enqueued
    assert np.all(out[0].cpu().numpy() == 9)
