"""gt_track_noalloc (tally workspace in the library's fixed per-GPU scratch
array) against gt_track through the C ABI: identical outputs on two calls in
a row, the second on a smaller input (fewer histories, fewer leaf instances),
so the second call runs over what the first left in the array; and the
documented rejections."""

import numpy as np
import pytest

from paper_2406_13849_amd import gt, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    gt.lib()
    yield


def _host(out):
    return dict(tally_fx=out.tally_fx.cpu().numpy().view(np.uint64), tally=out.tally.cpu().numpy(),
                seg_count=out.seg_count.cpu().numpy().view(np.uint32),
                seq_hash=out.seq_hash.cpu().numpy().view(np.uint64), end_code=out.end_code.cpu().numpy(),
                rec=None if out.rec is None else out.rec.cpu().numpy(), counters=out.counters_dict())


def _same(a, b, where):
    for k in ("tally_fx", "seg_count", "seq_hash", "end_code"):
        assert np.array_equal(a[k], b[k]), (where, k)
    # finalized tallies: the same fixed point converted the same way
    assert np.array_equal(a["tally"].view(np.int64), b["tally"].view(np.int64)), where
    if a["rec"] is not None:
        assert np.array_equal(a["rec"], b["rec"]), where
    assert a["counters"] == b["counters"], where
    assert a["counters"]["segments"] > 0, where


def test_noalloc_matches_gt_track_twice():
    import torch
    cases = [(2, 200_000, 500, 128, gt.PREC_MIXED), (1, 3_000, 50, 64, gt.PREC_FP64)]
    for cfg, n, rk, rc, prec in cases:
        fg = synth.make_config(cfg)
        G = gt.Geometry(fg)
        assert gt.track_workspace_bytes(G) <= gt.NOALLOC_SCRATCH_BYTES
        kw = dict(seed=synth.particle_seed(cfg) + 17, n_particles=n, geometry_id=cfg, precision=prec,
                  record_first_k=rk, record_cap=rc)
        print("noalloc: cfg%d, %d histories, precision %d" % (cfg, n, prec), flush=True)
        ref = gt.track(G, out=gt.alloc_outputs(G, n, rk, rc, workspace=True), **kw)
        torch.cuda.synchronize()
        out = gt.alloc_outputs(G, n, rk, rc)
        out.tally_fx.fill_(7)       # must be overwritten, not added to
        out.counters.fill_(3)
        gt.track_noalloc(G, out=out, **kw)
        torch.cuda.synchronize()
        _same(_host(ref), _host(out), "cfg%d" % cfg)
        G.close()


def test_noalloc_rejections():
    import ctypes as C
    import torch
    G = gt.Geometry(synth.make_config(1))
    # a workspace in the outputs is refused by the C ABI itself
    out = gt.alloc_outputs(G, 10, workspace=True)
    rc = gt.lib().gt_track_noalloc(G.h, C.byref(gt._params(1, 10)), C.byref(gt._out_struct(out)), None)
    assert rc == gt.GT_EINVAL and b"workspace" in gt.lib().gt_last_error()
    # a geometry whose workspace exceeds the fixed array: the three-level core
    # (2.86 M leaf instances); refused before any launch
    big = gt.Geometry(synth.make_config(3))
    assert gt.track_workspace_bytes(big) > gt.NOALLOC_SCRATCH_BYTES
    with pytest.raises(gt.GtError) as e:
        gt.track_noalloc(big, 1, 10, out=gt.alloc_outputs(big, 10))
    assert e.value.code == gt.GT_ECAPACITY
    torch.cuda.synchronize()
    big.close()
    G.close()
