"""The in-chip performance model of the trip kernel against the committed
counter measurements of the t = 1..8 sweep at 512^3 (no GPU): its geometry
reproduces the wave count, its instruction model the VALU and LDS counts,
its traffic model the HBM bytes, and its time the kernel durations."""

import json

from paper_1006_3148_amd import perfmodel as pm


def test_model_reproduces_counters_and_times():
    with open(pm.DEFAULT_DATA) as f:
        doc = json.load(f)
    params, rows = pm.report(pm.DEFAULT_DATA)
    for r, m in zip(rows, doc["rows"]):
        g = pm.geometry(512, m["t"], m["rows_per_wave"], m["waves"], m["seg_len"])
        assert g["waves"] == m["SQ_WAVES"]
        assert abs(r["valu_pred"] / r["valu_meas"] - 1) < 0.015, r
        if r["batched"]:
            # T writes and between T and 2T reads per wave and step (the
            # compiler pairs some of the batched reads)
            assert r["lds_pred_min"] * 0.995 <= r["lds_meas"] <= r["lds_pred"] * 1.005, r
        else:
            assert abs(r["lds_pred"] / r["lds_meas"] - 1) < 0.005, r
        assert abs(r["hbm_pred"] / r["hbm_meas"] - 1) < 0.06, r
        assert abs(r["time_pred_us"] / r["time_meas_us"] - 1) < 0.10, r
    # about 11 VALU instructions per cell-stage: 5 adds, 1 multiply, 4 DPP
    # moves and the pass-through selects
    assert 10.0 < params["valu"][0] < 12.0
