"""Tuning table (host side, no GPU): pcf_load_tuning validates and installs a
per-size-class policy table; pcf_policy_for and pcf_workspace_bytes follow it;
a bad file changes nothing."""
import json

import pytest


@pytest.fixture(scope="module")
def P():
    from paper_2405_07122_amd import pcfsort
    pcfsort.load()
    yield pcfsort
    pcfsort.pcf_load_tuning(None)


def _table(entries):
    return {"format": "pcfsort-tuning-1", "device": "test", "entries": entries}


def _entry(kt, pay, lo, hi, **pol):
    return {"key_type": kt, "with_payload": pay, "min_n": lo, "max_n": hi, "policy": pol}


def test_load_and_lookup(P, tmp_path):
    default = P.get_policy()
    f = tmp_path / "t.json"
    f.write_text(json.dumps(_table([
        _entry(0, 0, 0, 1 << 20, max_buckets=128, chunk_keys=8192),
        _entry(0, 0, 1 << 20, 1 << 32, max_buckets=512, target_child=4096),
        _entry(1, 1, 0, 1 << 32, samples_per_bucket=32),
    ])))
    ws_before = P.workspace_bytes(P.KEY_F64, 1 << 22)
    P.pcf_load_tuning(str(f))
    assert P.policy_for(P.KEY_F64, 1000)["max_buckets"] == 128
    assert P.policy_for(P.KEY_F64, 1000)["chunk_keys"] == 8192
    big = P.policy_for(P.KEY_F64, 1 << 22)
    assert big["max_buckets"] == 512 and big["target_child"] == 4096
    assert big["bins_per_bucket"] == default["bins_per_bucket"]  # omitted: default
    assert P.policy_for(P.KEY_U64, 5000, True)["samples_per_bucket"] == 32
    assert P.policy_for(P.KEY_U64, 5000, False) == default  # no entry of that kind
    # the workspace query follows the table (more buckets per node: larger)
    assert P.workspace_bytes(P.KEY_F64, 1 << 22) != ws_before
    P.pcf_load_tuning(None)
    assert P.policy_for(P.KEY_F64, 1 << 22) == default


@pytest.mark.parametrize("bad", [
    "not json",
    json.dumps({"format": "other", "entries": []}),
    json.dumps(_table([_entry(0, 0, 10, 5)])),                          # empty class
    json.dumps(_table([_entry(2, 0, 0, 10)])),                          # key type
    json.dumps(_table([_entry(0, 0, 0, 100, max_buckets=300)])),        # not a power of two
    json.dumps(_table([_entry(0, 0, 0, 100, lds_cap=100000)])),         # over the LDS limit
    json.dumps(_table([_entry(0, 0, 0, 100), _entry(0, 0, 50, 200)])),  # overlap
    json.dumps(_table([_entry(0, 0, 0, 100, tau=1.5)])),                # not an integer
])
def test_bad_files_are_rejected(P, tmp_path, bad):
    good = tmp_path / "good.json"
    good.write_text(json.dumps(_table([_entry(0, 0, 0, 1 << 32, max_buckets=64)])))
    P.pcf_load_tuning(str(good))
    f = tmp_path / "bad.json"
    f.write_text(bad)
    with pytest.raises(P.PcfError) as ei:
        P.pcf_load_tuning(str(f))
    assert ei.value.code == P.ERR_INVALID_ARGUMENT
    assert P.policy_for(P.KEY_F64, 1000)["max_buckets"] == 64  # unchanged
    P.pcf_load_tuning(None)


def test_missing_file(P):
    with pytest.raises(P.PcfError):
        P.pcf_load_tuning("/nonexistent/tuning.json")
