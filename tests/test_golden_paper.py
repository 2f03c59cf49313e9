"""The paper's printed push-rate table (Sec. 7, Table 3) transcribed in
tests/golden/paper_table3.json: its columns must agree with each other
(rate = 1/time), which pins the transcription.  The values are context for
bench.py, not targets."""
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def test_table3_columns_are_consistent():
    t = json.load(open(os.path.join(HERE, "golden", "paper_table3.json")))
    for order, ns_core, ns_cpu, r_core, r_cpu in t["rows"]:
        assert abs(1e3 / ns_cpu - r_cpu) / r_cpu < 0.01, order
        assert abs(ns_core / ns_cpu - 8.0) < 0.1, order  # 8 cores
        if order != 4:  # the printed order-4 per-core rate is garbled
            assert abs(1e3 / ns_core - r_core) / r_core < 0.01, order
    rates = [r[4] for r in t["rows"]]
    assert rates == sorted(rates, reverse=True)
