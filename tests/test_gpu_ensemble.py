"""Ensemble heuristics on the GPU (hb_model_load_ensemble) against the oracle.

Members share one architecture and are fused into one model: side-by-side
layer-1 tables, one grouped launch per matrix layer, a head combining the
member outputs (minimum, or sum in member order) before the output rule.
* The fused output equals the oracle's ensemble output (tolerances as for
  single networks) at FP32, BF16 and FP8, for both rules.
* The fused model's combined output equals the minimum / sum of the members
  evaluated as separate models, bitwise (each member's columns go through the
  same MFMA sequence).
* 8-puzzle: min-ensemble of two networks with min(., Manhattan): the h table on
  all 181,440 states equals the oracle's, and Batch IDA* counts equal the
  serial oracle's on that table.
* Manhattan plus summed residuals (combine_md = 3) follows the written-out rule.
"""
import numpy as np
import pytest

import oracle as O
import paper_2507_11916_amd as hb
import synth
from tests import layerwise

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {hb.HB_FP32: 1e-5, hb.HB_BF16: 2e-3, hb.HB_FP8_E4M3: 2e-2}


def _members(tmp_path, net, width, seeds, bias):
    paths = []
    for s in seeds:
        p = str(tmp_path / f"{net}_{width}_{s}.hbw")
        spec = synth.widened(net, width) if width else None
        synth.write_weights(p, net, seed=s, head_bias=bias, spec=spec)
        paths.append(p)
    return paths


def _y(model, packed):
    d_p = torch.from_numpy(np.ascontiguousarray(packed)).cuda()
    d_h = torch.zeros(packed.shape[0], dtype=torch.int32, device="cuda")
    d_y = torch.zeros(packed.shape[0], dtype=torch.float32, device="cuda")
    model.eval_batch(d_p, d_h, d_y)
    torch.cuda.synchronize()
    return d_h.cpu().numpy(), d_y.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("rule", [hb.HB_ENSEMBLE_MIN, hb.HB_ENSEMBLE_SUM])
@pytest.mark.parametrize("prec", [hb.HB_FP32, hb.HB_BF16, hb.HB_FP8_E4M3])
def test_ensemble_matches_oracle(tmp_path, prec, rule):
    paths = _members(tmp_path, "stp4_res", 256, [22, 23, 24], 40.0)
    st = synth.stp_walks(4, synth.throughput_seeds(300, 404), lengths=200)
    packed = hb.hb_encode(1, st)
    m = hb.Model(paths, prec=prec, out=hb.HB_OUT_REG_REAL, ensemble_rule=rule)
    members = [O.Net(p) for p in paths]
    scales = None
    if prec == hb.HB_FP8_E4M3:
        calib = synth.stp_walks(4, synth.throughput_seeds(1024, 4242), lengths=200)
        m.calibrate(torch.from_numpy(hb.hb_encode(1, calib)).cuda())
        fused = np.max([net.calibrate(calib) for net in members], axis=0)  # one scale per fused tensor
        np.testing.assert_array_equal(m.act_scales(), fused.astype(np.float32))
        scales = [fused] * len(members)
    # every member's stored activations, layer by layer (tests/layerwise.py)
    tf = layerwise.teacher_forced(m, members, st, torch.from_numpy(packed).cuda(), int(prec),
                                  None if scales is None else scales[0])
    _, y = _y(m, packed)
    # the fused head: the members' outputs on their own last activations, combined
    ys = np.stack([t[:, 0] for t in tf["y_tf"]])
    es = np.stack([e[:, 0] for e in tf["e_head"]])
    y_tf = ys.min(axis=0) if rule == hb.HB_ENSEMBLE_MIN else ys.sum(axis=0)
    e = (es.max(axis=0) if rule == hb.HB_ENSEMBLE_MIN else es.sum(axis=0)) + len(members) * layerwise.U * np.abs(ys).sum(axis=0)
    assert np.all(np.abs(y - y_tf) <= e), np.abs(y - y_tf).max()
    # whole forward pass: rows without a flip follow the oracle's quantised pass
    y_ref = O.ensemble_forward(members, st, rule, mode=int(prec), act_scales=scales)
    y_exact = O.ensemble_forward(members, st, rule)
    fl = tf["flip_rows"]
    assert np.all(np.abs(y - y_ref)[~fl] <= e[~fl] + 1e-9 * np.abs(y_ref[~fl]))
    scale = np.maximum(1.0, np.abs(y_ref))
    d = np.abs(y - y_ref) / scale
    env = np.abs(y_ref - y_exact) / scale
    assert np.all(d[fl] <= 2 * env[fl] + TOL[prec])
    print("ensemble prec", prec, "rule", rule, "per-layer", tf["stats"], "rows with a flip", fl.mean())


@pytest.mark.parametrize("prec,tile", [(hb.HB_FP32, 0), (hb.HB_BF16, 0), (hb.HB_BF16, 6), (hb.HB_BF16, 10),
                                       (hb.HB_FP32, 10), (hb.HB_BF16, 15), (hb.HB_FP32, 17)])
def test_fused_equals_separate_members(tmp_path, prec, tile):
    """The fused ensemble (grouped GEMMs: each member's columns read their own
    slice of the activations) equals the members evaluated one by one, for the
    automatic tile and forced ring, 8-wave and wide-block ring tiles."""
    paths = _members(tmp_path, "stp4_res", 256, [31, 32], 40.0)
    st = synth.stp_walks(4, synth.throughput_seeds(500, 505), lengths=200)
    packed = hb.hb_encode(1, st)

    def model(p, **kw):
        m = hb.Model(p, prec=prec, out=hb.HB_OUT_REG_REAL, **kw)
        if tile:
            m.set_tile(tile)
        return m

    ys = [_y(model(p), packed)[1] for p in paths]
    y_min = _y(model(paths, ensemble_rule=hb.HB_ENSEMBLE_MIN), packed)[1]
    y_sum = _y(model(paths, ensemble_rule=hb.HB_ENSEMBLE_SUM), packed)[1]
    np.testing.assert_array_equal(y_min, np.minimum(ys[0], ys[1]))
    np.testing.assert_array_equal(y_sum, (ys[0].astype(np.float32) + ys[1].astype(np.float32)).astype(np.float64))


def test_min_ensemble_8puzzle_search(tmp_path):
    paths = _members(tmp_path, "stp3_small", 0, [11, 12], 14.0)
    allst = O.all8()
    members = [O.Net(p) for p in paths]
    md = O.manhattan(0, allst)
    h_ref = O.h_regression(O.ensemble_forward(members, allst, O.ENS_MIN), md, combine=1)
    m = hb.Model(paths, prec=hb.HB_FP32, combine_md=1, max_batch=4096, ensemble_rule=hb.HB_ENSEMBLE_MIN)
    h, _ = _y(m, hb.hb_encode(0, allst))
    assert np.array_equal(h, h_ref), "h tables differ; counts cannot be compared"
    ranks = np.array([O.lib().orc_perm9_rank(np.ascontiguousarray(s).ctypes.data) for s in allst])
    table = np.zeros(362880, dtype=np.int32)
    table[ranks] = h_ref
    for i, s in enumerate(synth.stp3_instances(30)):
        p = hb.default_params(batch_size=64, work_num=4, complete_final_iter=1)
        r = hb.cbdfs_solve(0, s, model=m, combine=hb.HB_H_NN, threads=1 + 3 * (i % 2), params=p)
        o = O.ida(0, s, hkind=O.H_TABLE8, table8=table, complete_final=True)
        assert r["status"] == hb.HB_OK and r["cost"] == o["cost"]
        assert [(it["bound"], it["expanded"], it["generated"]) for it in r["iters"]] == \
               [(it["bound"], it["expanded"], it["generated"]) for it in o["iters"]]


def test_manhattan_plus_residual_rule(tmp_path):
    paths = _members(tmp_path, "stp4_res", 256, [41, 42], -4.0)  # summed residuals around 0-3
    st = synth.stp_walks(4, synth.throughput_seeds(400, 606), lengths=200)
    m = hb.Model(paths, prec=hb.HB_FP32, combine_md=3, ensemble_rule=hb.HB_ENSEMBLE_SUM)
    h, _ = _y(m, hb.hb_encode(1, st))
    members = [O.Net(p) for p in paths]
    y_ref = O.ensemble_forward(members, st, O.ENS_SUM)
    md = O.manhattan(1, st)
    h_ref = O.h_regression(y_ref, md, combine=3)
    fr = y_ref - np.floor(y_ref)
    amb = np.minimum(fr, 1 - fr) <= TOL[hb.HB_FP32] * np.maximum(1, np.abs(y_ref))
    assert np.all((h == h_ref) | amb)
    assert np.all(h >= md)
    assert (h > md).any() and (h == md).any()  # both sides of the clamp are exercised
