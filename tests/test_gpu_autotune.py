"""The project autotuner: it picks one of its candidate dispatches, records
it in the cache file, reuses the cached choice, and does not change H."""
import json
import sys

import pytest

import bse_synth as B

pytestmark = pytest.mark.gpu


def test_autotune_choice_cache_and_results(tmp_path):
    import paper_1206_3518_amd as P
    import torch
    systems = [
        B.make_system(B.cell_sc(10.0), (16, 16, 16), (2, 2, 2), 2, 2, 3.0, seed=51),
        B.make_system(B.cell_fcc(9.0), (16, 16, 16), (3, 1, 1), 1, 3, 2.0, seed=52),
    ]
    devs = [P.DeviceSystem(s) for s in systems]
    ws = P.workspace(P.bse_workspace_size(devs))
    P.bse_build_H(devs, P.BSE_FP64, 0, ws)
    torch.cuda.synchronize()
    before = [d.H.clone() for d in devs]
    cache = tmp_path / "tune.jsonl"
    got = P.bse_autotune(devs, P.BSE_FP64, cache, ws)
    tried = P.bse_autotune_last()
    print("autotune choice:", got, flush=True)
    sys.stdout.flush()
    pd = [t for t in tried if t["s1_ms"] == 0]
    assert len(pd) == 13 and sorted(t["order"] for t in pd if not t["persistent"]) == [0, 0, 0, 1, 1, 1, 2, 2, 2]
    assert got["order"] in (0, 1, 2) and (got["order"] == 0 or not got["persistent"])
    assert got["persistent"] in (0, 1) and got["pd_ms"] > 0.0
    if got["persistent"]:
        assert got["wg_per_cu"] in (1, 2, 3, 4)
    else:
        assert got["ktile"] in (4, 8, 16)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert (rec["persist"], rec["ktile"], rec["wg_per_cu"]) == (got["persistent"], got["ktile"], got["wg_per_cu"])
    # a second call takes the cached line without timing again
    again = P.bse_autotune(devs, P.BSE_FP64, cache, ws)
    assert {k: again[k] for k in ("persistent", "ktile", "wg_per_cu")} == \
        {k: got[k] for k in ("persistent", "ktile", "wg_per_cu")}
    assert abs(again["pd_ms"] - got["pd_ms"]) <= 1e-6 * got["pd_ms"]
    assert len(cache.read_text().splitlines()) == 1
    # builds after tuning give the same H, bit for bit
    for d in devs:
        d.H.zero_()
    P.bse_build_H(devs, P.BSE_FP64, 0, ws)
    torch.cuda.synchronize()
    for d, h in zip(devs, before):
        assert torch.equal(d.H, h)


def test_autotune_fp32_pairdens_separate_key(tmp_path):
    """Tuning the FP32 pair-density kernel writes its own cache line and leaves
    the FP64 build unchanged; the FP32 build after tuning is bit-identical to
    the one before (the dispatch changes the order, not the arithmetic)."""
    import paper_1206_3518_amd as P
    import torch
    s = B.make_system(B.cell_sc(10.0), (16, 16, 16), (2, 2, 2), 2, 2, 3.0, seed=53)
    d = P.DeviceSystem(s)
    ws = P.workspace(P.bse_workspace_size([d], P.BSE_BF16X3, P.BSE_FP32_PAIRDENS))
    P.bse_build_H([d], P.BSE_BF16X3, P.BSE_FP32_PAIRDENS, ws)
    torch.cuda.synchronize()
    before = d.H.clone()
    cache = tmp_path / "tune.jsonl"
    P.bse_autotune([d], P.BSE_BF16X3, cache, ws)
    got = P.bse_autotune([d], P.BSE_BF16X3, cache, ws, flags=P.BSE_FP32_PAIRDENS)
    print("FP32 autotune choice:", got, flush=True)
    lines = [json.loads(x) for x in cache.read_text().splitlines()]
    assert len(lines) == 2 and lines[0]["key"] != lines[1]["key"] and "f32" in lines[1]["key"]
    d.H.zero_()
    P.bse_build_H([d], P.BSE_BF16X3, P.BSE_FP32_PAIRDENS, ws)
    torch.cuda.synchronize()
    assert torch.equal(d.H, before)
    with pytest.raises(P.BseError):
        P.bse_autotune([d], P.BSE_FP64, None, ws, flags=P.BSE_FP32_PAIRDENS)


@pytest.mark.parametrize("prec", ["fp64", "split_fp32", "bf16x3"])
def test_stage1_tile_shapes(tmp_path, prec):
    """The autotuner times the first direct-term contraction with 64- and
    (BF16 parts) 128-row tiles; a cached choice of either shape gives H
    bit-identical to the default build (each output element sums its products
    in the same order whatever the tile)."""
    import paper_1206_3518_amd as P
    import torch
    p = P.PRECISIONS[prec]
    s = B.make_config(1)
    d = P.DeviceSystem(s)
    ws = P.workspace(P.bse_workspace_size([d], p))
    P.bse_build_H([d], p, 0, ws)
    torch.cuda.synchronize()
    before = d.H.clone()
    cache = tmp_path / "tune.jsonl"
    got = P.bse_autotune([d], p, cache, ws)
    tried = P.bse_autotune_last()
    s1 = {t["s1_rows"]: t["s1_ms"] for t in tried if t["s1_ms"] > 0}
    print(f"{prec}: stage-1 tiles {s1}, chosen {got['s1_rows']}", flush=True)
    shapes = {64, 128} if prec == "bf16x3" else {64}  # FP64 and FP32 parts: 64-row tiles only
    assert set(s1) == shapes and got["s1_rows"] in shapes and got["s1_ms"] == min(s1.values())
    line = json.loads(cache.read_text().splitlines()[0])
    for rows in sorted(shapes, reverse=True):
        line["s1_rows"] = rows
        cache.write_text(json.dumps(line) + "\n")
        assert P.bse_autotune([d], p, cache, ws)["s1_rows"] == rows
        d.H.zero_()
        P.bse_build_H([d], p, 0, ws)
        torch.cuda.synchronize()
        assert torch.equal(d.H, before)
