"""hb_eval_batch_noalloc against hb_eval_batch, through the C ABI.

The allocation-free entry point runs the same kernels with its activation
buffers in the library's fixed device array, so its outputs must be bitwise
equal to hb_eval_batch's.  Two calls in a row, the second on fewer states,
check that nothing from the first call leaks into the second (the array keeps
the last call's contents).  Sizes beyond the array's limit are rejected.
"""
import numpy as np
import pytest

import paper_2507_11916_amd as hb
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _run(fn, d_packed, n, n_out):
    d_h = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    d_y = torch.full((n * n_out,), float("nan"), dtype=torch.float32, device="cuda")
    fn(d_packed[:n], d_h, d_y)
    torch.cuda.synchronize()
    return d_h.cpu().numpy(), d_y.cpu().numpy()


def _cube_states(count):
    mv = synth.rc_walk_moves_array(synth.throughput_seeds(count, 9009), length_base=20, length_span=11)
    return hb.hb_apply_moves(2, mv)


CASES = [
    ("stp4_res", hb.HB_FP32, hb.HB_OUT_REG_FLOOR, 1),
    ("stp4_res", hb.HB_BF16, hb.HB_OUT_REG_FLOOR, 1),
    ("stp4_res", hb.HB_FP8_E4M3, hb.HB_OUT_REG_FLOOR, 1),
    ("rc_cls", hb.HB_BF16, hb.HB_OUT_CLS_QUANTILE, 21),
]


@pytest.mark.parametrize("name,prec,out,n_out", CASES)
def test_noalloc_equals_eval_batch_on_two_calls(net_files, name, prec, out, n_out):
    dom = 2 if name == "rc_cls" else 1
    sizes = (1500, 333)  # the second call is smaller: ragged tails, several tiles
    st = _cube_states(sizes[0]) if dom == 2 else synth.stp_walks(4, synth.throughput_seeds(sizes[0]), lengths=200)
    d_packed = _dev(hb.hb_encode(dom, st))
    m = hb.Model(net_files[name], prec=prec, out=out, q=0.99, combine_md=(dom == 1))
    if prec == hb.HB_FP8_E4M3:
        m.calibrate(d_packed)
    for n in sizes:
        h_ref, y_ref = _run(m.eval_batch, d_packed, n, n_out)
        h, y = _run(m.eval_batch_noalloc, d_packed, n, n_out)
        np.testing.assert_array_equal(h, h_ref)
        np.testing.assert_array_equal(y.view(np.uint32), y_ref.view(np.uint32))
        assert np.all(h >= 0)
    m.close()


def test_noalloc_rejects_sizes_beyond_its_array(net_files):
    m = hb.Model(net_files["stp4_res"], prec=hb.HB_FP32, max_batch=16384)
    n = 8192 + 1  # two FP32 rows of 1024 elements per state: 8192 states fill 64 MiB
    d_packed = torch.zeros(n * 8, dtype=torch.uint8, device="cuda").view(n, 8)
    d_h = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(hb.HBError) as e:
        m.eval_batch_noalloc(d_packed, d_h)
    assert e.value.status == hb.HB_E_INVAL and "allocation-free limit" in str(e.value)
    m.close()
