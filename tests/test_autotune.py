"""The tuning table's host side (no GPU): put / get / replace / clear and
the JSON cache round trip of paper_1911_03813_amd.autotune."""

import json

import pytest

import paper_1911_03813_amd as S
from paper_1911_03813_amd import autotune as AT


@pytest.fixture(autouse=True)
def empty_table():
    AT.clear()
    yield
    AT.clear()


def _entry(**kw):
    e = dict(kind=AT.KIND_FG, prec=S.PREC_FP64, n_bucket=10, p_bucket=17, r_bucket=7, v0=128, v1=32, us=812.5)
    e.update(kw)
    return e


def test_put_get_replace_clear():
    assert AT.entries() == []
    AT.put(_entry())
    AT.put(_entry(kind=AT.KIND_GROUPED, v0=8, v1=0))
    assert len(AT.entries()) == 2
    AT.put(_entry(v0=64))                     # same key: replaced
    got = AT.entries()
    assert len(got) == 2 and got[0]["v0"] == 64 and got[1]["kind"] == AT.KIND_GROUPED
    AT.clear()
    assert AT.entries() == []


def test_bad_entries_are_refused():
    with pytest.raises(S.SymtdError):
        AT.put(_entry(kind=7))
    with pytest.raises(S.SymtdError):
        AT.put(_entry(v0=-1))


def test_json_round_trip(tmp_path):
    AT.put(_entry())
    AT.put(_entry(kind=AT.KIND_GROUPED, n_bucket=6, p_bucket=12, r_bucket=6, v0=32, v1=0, us=41.0))
    path = tmp_path / "cache.json"
    AT.save(str(path), {"device": "test"})
    doc = json.loads(path.read_text())
    assert doc["meta"]["device"] == "test" and len(doc["entries"]) == 2
    AT.clear()
    assert AT.load(str(path)) == 2
    assert AT.entries() == doc["entries"]


def test_buckets_are_ceil_log2():
    assert [AT.bucket(x) for x in (1, 2, 3, 4, 5, 1000, 1024, 1025, 100_000)] == [0, 1, 2, 2, 3, 10, 10, 11, 17]
