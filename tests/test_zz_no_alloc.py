"""The allocation-free batch fit (sb_fit_batch_noalloc, through the C ABI) against the allocating
one (sb_fit_batch) on the same inputs: bitwise equal results on two calls in a row, the second on
a smaller batch (the fixed state array keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from gpu_util import torch_or_skip

pytestmark = pytest.mark.gpu


def _items(o6, n, k):
    out = []
    for r in synth.fit_requests(n, k=k):
        b = synth.Batch(np.float32([r.z]), np.float32([r.theta_true[0]]), np.float32([r.theta_true[1]]),
                        np.float32([r.theta_true[2]]), np.float32([r.theta_true[3]]), r.t, r.band,
                        np.int32([0, len(r.t)]))
        d, sig, w = synth.make_data(o6.bandflux(b), b.sn_offsets, r.normals)
        out.append((r, d, sig, w))
    return out


def _device(torch, items, free):
    dv = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dt)).cuda()
    n = np.array([len(r.t) for r, *_ in items])
    off = np.zeros(len(items) + 1, np.int32)
    off[1:] = np.cumsum(n)
    th = np.array([r.theta_init for r, *_ in items], np.float64)
    return dict(z=dv([r.z for r, *_ in items], np.float32), t0=dv(th[:, 0], np.float32),
                x0=dv(th[:, 1], np.float32), x1=dv(th[:, 2], np.float32), c=dv(th[:, 3], np.float32),
                t=dv(np.concatenate([r.t for r, *_ in items]), np.float32),
                band=dv(np.concatenate([r.band for r, *_ in items]), np.int32), fit_offsets=dv(off, np.int32),
                data=dv(np.concatenate([d for _, d, _, _ in items]), np.float32),
                inv_sigma2=dv(np.concatenate([w for *_, w in items]), np.float32), free_mask=dv(free, np.int32))


def test_noalloc_batch_fit_matches_the_allocating_call(model, bands6):
    torch = torch_or_skip()
    from paper_2504_08081_amd import saltbf as sb
    o6 = oracle.Oracle(model, bands6)
    ctx = sb.Context.from_model(model, bands6)
    L = sb.lib()
    big = _items(o6, 48, 61)
    small = _items(o6, 17, 62)
    for step, items in enumerate((big, small)):
        free = np.array([(0, 7, 13, 15)[i % 4] for i in range(len(items))], np.int32)
        d = _device(torch, items, free)
        print(f"case: sb_fit_batch_noalloc call {step}, {len(items)} fits", flush=True)
        ref = ctx.fit_batch(**d)
        desc = ctx._fit_batch_desc(**d)
        out = torch.full((len(items), sb.FIT_OUT_WORDS), -1, dtype=torch.int32, device="cuda")
        st = L.sb_fit_batch_noalloc(ctx._h, ctypes.byref(desc), ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == sb.SB_OK, L.sb_last_error()
        torch.cuda.synchronize()
        ctx.device_check()
        assert torch.equal(out, ref), step
        res = sb.fit_results(out)
        assert np.all(res["status"] == sb.SB_OK) and np.all(res["iters"] == 50)
    # a batch beyond the fixed array is refused before anything is launched
    desc = ctx._fit_batch_desc(**_device(torch, small, np.zeros(len(small), np.int32)))
    desc.n_fit = sb.SB_FIT_NOALLOC_MAX + 1
    assert L.sb_fit_batch_noalloc(ctx._h, ctypes.byref(desc), ctypes.c_void_p(1), None) == sb.SB_ERR_ARG
    assert b"SB_FIT_NOALLOC_MAX" in L.sb_last_error()
    ctx.close()
