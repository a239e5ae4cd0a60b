"""Host-side pieces of bench.py (no GPU): the CLI parses its defaults, every leg the default run
calls exists, the algorithmic byte count follows its formula, the counter summary lookup, and
the oracle baseline on a tiny budget."""

import json
import sys

import bench


def test_default_run_entry_points_exist(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert a.gpus == 1 and a.steps > 0 and a.warmup >= 0
    for name in ("cpu_baseline", "accuracy_reference", "accuracy_leg", "uneven_leg", "tv_leg",
                 "measured_traffic", "step_percentiles", "time_loop", "main"):
        assert callable(getattr(bench, name)), name


def test_algorithmic_bytes_formula():
    class Info:
        nnz, n_polar, n_cart, cols_touched, polar_nonempty = 100, 10, 20, 15, 9
    fwd, adj = bench.algorithmic_bytes(Info, 2, 4)
    assert fwd == 100 * 6 + 4 * 11 + 32 * (15 + 10)
    assert adj == 100 * 6 + 4 * 21 + 32 * (9 + 20)


def test_counter_summary_matches_sources_or_is_ignored():
    import paper_2003_12677_amd as tomo
    t = tomo.Operator(8, 6, 9, device=-1).get_tuning()
    r = bench.measured_traffic("spmm_adj_bf16", t)
    with open(bench.COUNTERS) as fh:
        c = json.load(fh)
    if c["source_sha256"] == bench.source_digest(t):
        assert r is not None and r["total_bytes"] > 0
    else:
        assert r is None
    assert bench.measured_traffic("spmm_adj_bf16", dict(t, adj_sell_max=-1)) is None
