"""GPU tests of the output rules that the seeded networks rarely reach: exact
halves under round-half-even, tied logits under arg-max, non-finite outputs,
and the host-side min with the classic heuristic inside cbdfs_solve.

The networks are hand-built with outputs known in closed form (tests/nets.py:
y = 2 MD - 2 off the goal, exact in float32 and bfloat16), so the expected h
is written out here and also checked against the oracle's rule.
"""
import numpy as np
import pytest

import oracle as O
import paper_2507_11916_amd as hb
import synth
from tests import nets

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _eval(model, states, domain, n_out):
    d_p = torch.from_numpy(hb.hb_encode(domain, states)).cuda()
    d_h = torch.zeros(len(states), dtype=torch.int32, device="cuda")
    d_y = torch.zeros(len(states) * n_out, dtype=torch.float32, device="cuda")
    model.eval_batch(d_p, d_h, d_y)
    torch.cuda.synchronize()
    return d_h.cpu().numpy(), d_y.cpu().numpy().reshape(-1, n_out)


def _reg_net(path, shift, bias_nan=False):
    """One output y = 2 MD - 2 + shift (8-puzzle)."""
    ts = [np.asarray(t, dtype=np.float64) for t in nets.md_net_tensors(3)]
    ts[-2] = ts[-2][:, 1:2]
    ts[-1] = np.asarray(ts[-1]).reshape(-1)[1:2] + shift
    if bias_nan:
        ts[-1] = np.array([np.nan])
    synth.write_weights_arrays(path, 0, 81, [2, 3], 1, 1, 0, ts)


def _cls_net(path, nan_logit=False):
    """Three logits (2 MD - 2, 2 MD - 2, 10): a three-way tie at MD = 6."""
    ts = [np.asarray(t, dtype=np.float64) for t in nets.md_net_tensors(3)]
    ts[-2] = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 1.0, 0.0]])
    ts[-1] = np.array([-1.0, -1.0, np.nan if nan_logit else 10.0])
    synth.write_weights_arrays(path, 0, 81, [2, 3], 1, 3, 1, ts)


@pytest.fixture(scope="module")
def states8():
    st = O.all8()
    md = O.manhattan(0, st)
    return st[md >= 1], md[md >= 1]  # the closed form holds off the goal


@pytest.mark.parametrize("prec", [hb.HB_FP32, hb.HB_BF16])
@pytest.mark.parametrize("shift,offset", [(0.5, 0.0), (-0.5, 0.0), (0.5, 1.0), (0.25, 0.0)])
def test_round_half_even_on_exact_halves(tmp_path, states8, prec, shift, offset):
    st, md = states8
    path = str(tmp_path / "r.hbw")
    _reg_net(path, shift)
    m = hb.Model(path, prec=prec, out=hb.HB_OUT_REG_ROUND, offset=offset)
    h, y = _eval(m, st, 0, 1)
    np.testing.assert_array_equal(y[:, 0], 2.0 * md - 2 + shift - offset)  # raw = y - offset, exact
    v = 2 * md - 2 + shift - offset
    expect = np.maximum(0, np.where(v - np.floor(v) == 0.5, 2 * np.round(v / 2), np.round(v))).astype(np.int32)
    if shift in (0.5, -0.5):  # every value is a half: ties go to the even neighbour, 2 MD - 2 (or its offset)
        assert np.all(v - np.floor(v) == 0.5)
        np.testing.assert_array_equal(expect % 2, 0)
    np.testing.assert_array_equal(h, expect)
    np.testing.assert_array_equal(h, O.h_regression(2.0 * md - 2 + shift, None, offset=offset, mode=1))
    m.close()


@pytest.mark.parametrize("prec", [hb.HB_FP32, hb.HB_BF16])
def test_argmax_takes_the_lowest_index_on_ties(tmp_path, states8, prec):
    st, md = states8
    path = str(tmp_path / "c.hbw")
    _cls_net(path)
    m = hb.Model(path, prec=prec, out=hb.HB_OUT_CLS_ARGMAX)
    h, z = _eval(m, st, 0, 3)
    np.testing.assert_array_equal(z, np.stack([2.0 * md - 2, 2.0 * md - 2, np.full(md.size, 10.0)], axis=1))
    expect = np.where(md >= 6, 0, 2)  # 2 MD - 2 >= 10 ties class 0 with class 1 (and class 2 at MD = 6)
    assert (md == 6).any() and (md > 6).any() and (md < 6).any()
    np.testing.assert_array_equal(h, expect)
    np.testing.assert_array_equal(h, O.Net(path).h(z.astype(np.float64), 4))
    m.close()


def test_non_finite_outputs_fall_back(tmp_path, states8):
    st, md = states8
    path = str(tmp_path / "nan.hbw")
    _reg_net(path, 0.0, bias_nan=True)
    for combine_md, expect in ((True, md), (False, np.zeros_like(md))):
        m = hb.Model(path, prec=hb.HB_FP32, combine_md=combine_md)
        h, y = _eval(m, st, 0, 1)
        assert np.all(np.isnan(y[:, 0]))
        np.testing.assert_array_equal(h, expect)
        np.testing.assert_array_equal(h, O.Net(path).h(y.astype(np.float64), 0, classic=md if combine_md else None))
        m.close()
    cpath = str(tmp_path / "nan_cls.hbw")
    _cls_net(cpath, nan_logit=True)
    for out in (hb.HB_OUT_CLS_QUANTILE, hb.HB_OUT_CLS_ARGMAX):
        m = hb.Model(cpath, prec=hb.HB_FP32, out=out, q=0.99)
        h, z = _eval(m, st, 0, 3)
        assert np.all(np.isnan(z[:, 2]))
        np.testing.assert_array_equal(h, 0)
        np.testing.assert_array_equal(h, O.Net(cpath).h(z.astype(np.float64), 3 if out == hb.HB_OUT_CLS_QUANTILE else 4))
        m.close()


def test_min_nn_classic_inside_cbdfs_solve(net_files):
    """HB_H_MIN_NN_CLASSIC: the network alone on the GPU (no Manhattan rule in
    the model), the min with Manhattan distance taken by the batch thread.  The
    GPU's unclamped table is checked on all 181,440 states first; then counts
    per iteration equal the oracle's IDA* with min(h_net, MD)."""
    path = net_files["stp3_small"]
    allst = O.all8()
    net = O.Net(path)
    h_net = net.h(net.forward(allst), 0)
    md = O.manhattan(0, allst)
    m = hb.Model(path, prec=hb.HB_FP32, max_batch=4096)
    h_gpu, _ = _eval(m, allst, 0, 1)
    assert np.array_equal(h_gpu, h_net), "h tables differ; counts cannot be compared"
    assert np.any(h_net > md) and np.any(h_net < md)  # both sides of the min occur
    ranks = O.perm9_rank(allst)
    table = np.zeros(362880, dtype=np.int32)
    table[ranks] = np.minimum(h_net, md)
    bfs, _ = O.bfs8()
    for i, s in enumerate(synth.stp3_instances(30)):
        p = hb.default_params(batch_size=64, work_num=4, complete_final_iter=1)
        r = hb.cbdfs_solve(0, s, model=m, combine=hb.HB_H_MIN_NN_CLASSIC, classic=hb.HB_CLASSIC_MD,
                           threads=1 + 3 * (i % 2), params=p)
        o = O.ida(0, s, hkind=O.H_TABLE8, table8=table, complete_final=True)
        assert r["status"] == hb.HB_OK and r["cost"] == o["cost"] == bfs[O.perm9_rank(s[None])[0]]
        assert [(it["bound"], it["expanded"], it["generated"]) for it in r["iters"] if it["complete"]] == \
               [(it["bound"], it["expanded"], it["generated"]) for it in o["iters"] if it["complete"]]
    m.close()


def test_real_valued_search_rejects_a_manhattan_rule(tmp_path):
    path = str(tmp_path / "r.hbw")
    _reg_net(path, 0.0)
    m = hb.Model(path, prec=hb.HB_FP32, out=hb.HB_OUT_REG_REAL, combine_md=True)
    r = hb.cbdfs_solve(0, synth.stp3_instances(1)[0], model=m, combine=hb.HB_H_NN_REAL, threads=1,
                       raise_on_error=False)
    assert r["status"] == hb.HB_E_INVAL
    m.close()
