"""hdm_matvec_noalloc (the allocation-free product) against hdm_matvec, through the C ABI.

Two calls in a row on the shared scratch array, the second with a smaller
input, then a half-precision operator with 16 columns and the normalised
product; each result must equal hdm_matvec's bit for bit (the same kernels in
the same order).  An operator whose workspace exceeds the array is refused,
with its output untouched, while hdm_matvec takes the same request.
"""
import ctypes as C

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _hdm():
    from paper_2311_06115_amd import hdm
    return hdm


def _op(name, **over):
    hdm = _hdm()
    cfg = synth.get_config(name)
    cfg.update(over)
    X, eps = synth.configs.make_inputs(cfg, cfg["n"])
    print(f"[gpu] noalloc: compress {name} n={cfg['n']} near={cfg['near_prec']}", flush=True)
    return hdm.Operator(torch.from_numpy(X).cuda(), eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"],
                        near_prec=cfg["near_prec"], far_prec=cfg["far_prec"])


def _both(op, nrhs, normalised, seed):
    hdm = _hdm()
    rng = np.random.default_rng(seed)
    x = torch.from_numpy(rng.standard_normal((nrhs, op.n))).cuda().contiguous()
    ref = torch.empty_like(x)
    out = torch.full_like(x, np.nan)
    hdm.check(hdm.lib().hdm_matvec(op.h, int(normalised), C.c_void_p(x.data_ptr()), C.c_void_p(ref.data_ptr()),
                                   nrhs, hdm._stream(torch)))
    hdm.check(hdm.lib().hdm_matvec_noalloc(op.h, int(normalised), C.c_void_p(x.data_ptr()),
                                           C.c_void_p(out.data_ptr()), nrhs, hdm._stream(torch)))
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_equals_matvec_two_calls_then_smaller():
    big = _op("scurve-32k")                 # float32 tiles, 32768 points
    small = _op("scurve-2k")                # float64 tiles, 2048 points
    ref, out = _both(big, 3, False, 1)
    assert np.array_equal(ref, out)
    ref, out = _both(small, 1, True, 2)     # second call: a smaller input on the same array
    assert np.array_equal(ref, out)
    ref, out = _both(big, 1, True, 3)       # and back: nothing stale from the smaller call
    assert np.array_equal(ref, out)
    big.close()
    small.close()


def test_noalloc_half_precision_block():
    op = _op("scurve-100k", n=20000, m=512)   # packed float16 near tiles on the matrix cores
    ref, out = _both(op, 16, False, 4)
    assert np.array_equal(ref, out)
    ref, out = _both(op, 5, True, 5)
    assert np.array_equal(ref, out)
    op.close()


def test_noalloc_refuses_an_operator_above_the_array():
    hdm = _hdm()
    # 100000 points on float32 near tiles: the near field's partial sums alone
    # take far more than 64 MiB, even for one column
    op = _op("scurve-100k", near_prec="f32")
    x = torch.zeros((1, op.n), dtype=torch.float64, device="cuda")
    y = torch.full_like(x, np.nan)
    st = hdm.lib().hdm_matvec_noalloc(op.h, 0, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), 1,
                                      hdm._stream(torch))
    assert st == 2 and b"MiB" in hdm.lib().hdm_last_error()
    torch.cuda.synchronize()
    assert torch.isnan(y).all()             # the output is untouched
    # the allocating product takes the same request
    hdm.check(hdm.lib().hdm_matvec(op.h, 0, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), 1,
                                   hdm._stream(torch)))
    torch.cuda.synchronize()
    assert torch.isfinite(y).all()
    op.close()
