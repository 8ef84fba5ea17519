"""Autotuner bookkeeping (no GPU): classes, table lookup, defaults."""
import json

from paper_1710_03647_amd import synth, tune


def test_graph_class_buckets():
    assert tune.graph_class(1 << 20, 16 << 20, 32) == "n2^20-d2^4-v32"
    assert tune.graph_class(1000, 4000, 32) == "n2^9-d2^2-v32"


def test_defaults_when_untuned(tmp_path):
    g = synth.gen_plain()
    assert tune.config_for(g, path=str(tmp_path / "none.json")) == tune.DEFAULTS


def test_table_lookup(tmp_path):
    g = synth.gen_plain()
    key = f"{tune.arch()}:{tune.graph_class(g.n, g.m, 32)}"
    p = tmp_path / "t.json"
    p.write_text(json.dumps({key: {"config": {"blocks_per_cu": 4, "dense_div": 8, "small_limit": 512,
                                              "partition": 1}}}))
    assert tune.config_for(g, path=str(p))["small_limit"] == 512


def test_proxy_is_smaller_instance_of_same_class():
    g = synth.gen_uniform(1 << 16, 8, 100, 3)
    proxy, rounds = tune._proxy(g)
    assert proxy.n == (1 << 12) and rounds == 0
