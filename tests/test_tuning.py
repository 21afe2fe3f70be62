"""Tuning table on the CPU: lookup by (precision, N bucket, L bucket), the
built-in default where the table has no entry or no table is loaded,
rejection of malformed files (the table is then unchanged), forcing, and
the committed table for gfx950.  Host only: nothing here touches a device."""
import json
import os

import pytest

from paper_1302_4000_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COMMITTED = os.path.join(ROOT, "paper_1302_4000_amd", "tuning", "gfx950.json")
DEFAULT = {"products": 3, "schedule": "staged", "band": 16, "frame": 1, "source": "default",
           "bucket": -1}


@pytest.fixture(scope="module", autouse=True)
def lib():
    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    binding.lib()
    yield
    binding.force_config(None)
    binding.load_tuning(None)


def table(entries, arch="gfx950", n_edges=(2, 256, 1024), l_edges=(1, 128)):
    return {"arch": arch, "n_edges": list(n_edges), "l_edges": list(l_edges),
            "entries": entries}


def write(tmp_path, obj, name="t.json"):
    p = tmp_path / name
    p.write_text(obj if isinstance(obj, str) else json.dumps(obj))
    return str(p)


def entry(prec, nb, lb, products=3, schedule="staged", band=16, frame=None, call=None):
    e = {"precision": prec, "n_bucket": nb, "l_bucket": lb, "products": products,
         "schedule": schedule, "band": band, "ms": {"ignored": 1.0}}
    if frame is not None:
        e["frame"] = frame
    if call is not None:
        e["call"] = call
    return e


def test_no_table_gives_default():
    binding.load_tuning(None)
    assert binding.tuning_path() == ""
    for prec in ("fp32", "bf16", "fp16"):
        assert binding.get_config(20000, 150, prec) == DEFAULT
    assert binding.get_config(20000, 150, "bf16x4")["products"] == 4


def test_lookup_by_bucket(tmp_path):
    t = table([entry("split_bf16", 0, 0, 4, "persistent", 8, frame=0),
               entry("split_bf16", 2, 1, 4, "staged", 32),
               entry("fp32", 1, 1, 3, "persistent", 24, frame=1),
               entry("split_fp16", 2, 0, 3, "staged", 8, frame=0)])
    binding.load_tuning(write(tmp_path, t))
    assert binding.tuning_path().endswith("t.json")
    # bucket 0 of N: [2, 256); bucket 0 of L: [1, 128)
    c = binding.get_config(100, 50, "bf16")
    assert c == {"products": 4, "schedule": "persistent", "band": 8, "frame": 0,
                 "source": "table", "bucket": 0}
    assert binding.get_config(255, 127, "bf16")["band"] == 8
    # edges are inclusive lower bounds; the last bucket is open
    assert binding.get_config(256, 127, "bf16") == DEFAULT          # (1, 0): no entry
    c = binding.get_config(10 ** 6, 10 ** 4, "bf16")
    assert (c["products"], c["band"], c["bucket"], c["frame"]) == (4, 32, 2 * 2 + 1, 1)
    c = binding.get_config(1024, 128, "fp32")
    assert c["schedule"] == "staged" and c["source"] == "default"   # fp32 entry is (1, 1)
    c = binding.get_config(300, 300, "fp32")
    assert (c["schedule"], c["band"], c["source"]) == ("persistent", 24, "table")
    # the persistent schedule drops the reference frame; the staged one keeps the table's
    assert binding.get_config(300, 300, "fp32")["frame"] == 0
    c = binding.get_config(5000, 100, "fp16")
    assert (c["schedule"], c["band"], c["frame"], c["source"]) == ("staged", 8, 0, "table")
    # precisions without a choice of products report their own count
    assert binding.get_config(300, 300, "fp16") == DEFAULT
    assert binding.get_config(100, 50, "bf16x4")["products"] == 4


@pytest.mark.parametrize("bad", [
    "{not json",
    json.dumps({"n_edges": [2], "l_edges": [1], "entries": []}),                 # no arch
    json.dumps(table([entry("split_bf16", 0, 0, products=5)])),                  # products
    json.dumps(table([entry("split_bf16", 3, 0)])),                              # bucket range
    json.dumps(table([entry("split_bf16", 0, 0, schedule="other")])),
    json.dumps(table([entry("split_bf16", 0, 0, schedule="looped")])),
    json.dumps(table([entry("split_bf16", 0, 0, band=0)])),
    json.dumps(table([entry("split_bf16", 0, 0, frame=2)])),
    json.dumps(table([entry("split_bf16", 0, 0, call="sometimes")])),
    json.dumps(table([entry("split_bf16", 0, 0, call=1)])),
    json.dumps(table([entry("fp64", 0, 0)])),                                    # no tile kernel
    json.dumps(table([], n_edges=(256, 2))),                                     # not ascending
    json.dumps(table([{"precision": "fp32", "n_bucket": 0}])),                   # incomplete
])
def test_malformed_table_rejected_and_table_unchanged(tmp_path, bad):
    good = table([entry("split_bf16", 0, 0, 4, "persistent", 8)])
    binding.load_tuning(write(tmp_path, good, "good.json"))
    before = binding.get_config(100, 50, "bf16")
    with pytest.raises(binding.ClucsoError) as ei:
        binding.load_tuning(write(tmp_path, bad, "bad.json"))
    assert ei.value.status == binding.ERR_INVALID_ARG
    assert binding.get_config(100, 50, "bf16") == before
    assert binding.tuning_path().endswith("good.json")


def test_batched_entries(tmp_path):
    """Batched calls take a bucket's "batched" entry, single calls its
    single-call entry (in either order in the file); a bucket without a
    batched entry gives batched calls its single-call entry, and one with
    only a batched entry gives single calls the built-in default."""
    t = table([entry("split_bf16", 0, 0, 3, "staged", 16, frame=1, call="batched"),
               entry("split_bf16", 0, 0, 4, "persistent", 8, frame=0),
               entry("split_bf16", 1, 0, 4, "staged", 8, frame=0, call="single"),
               entry("split_bf16", 1, 0, 3, "staged", 32, frame=1, call="batched"),
               entry("split_bf16", 2, 0, 4, "staged", 24, frame=0),
               entry("fp32", 0, 0, 3, "staged", 8, frame=1, call="batched")])
    binding.load_tuning(write(tmp_path, t))
    single = binding.get_config(100, 50, "bf16")
    batched = binding.get_config(100, 50, "bf16", batched=True)
    assert (single["products"], single["schedule"], single["band"], single["frame"]) == \
        (4, "persistent", 8, 0)
    assert (batched["products"], batched["schedule"], batched["band"], batched["frame"]) == \
        (3, "staged", 16, 1)
    assert single["bucket"] == batched["bucket"] == 0
    assert batched["source"] == "table"
    c = binding.get_config(300, 50, "bf16")
    assert (c["products"], c["band"], c["frame"]) == (4, 8, 0)
    c = binding.get_config(300, 50, "bf16", batched=True)
    assert (c["products"], c["band"], c["frame"]) == (3, 32, 1)
    # no batched entry: the single-call entry
    assert binding.get_config(5000, 50, "bf16", batched=True) == binding.get_config(5000, 50, "bf16")
    assert binding.get_config(5000, 50, "bf16")["band"] == 24
    # only a batched entry: single calls get the default
    assert binding.get_config(100, 50, "fp32") == DEFAULT
    assert binding.get_config(100, 50, "fp32", batched=True)["band"] == 8
    # no table: the default for both
    binding.load_tuning(None)
    assert binding.get_config(100, 50, "bf16", batched=True) == DEFAULT
    # forcing applies to both
    binding.load_tuning(write(tmp_path, t))
    binding.force_config(4, "staged", 12, frame=0)
    try:
        assert binding.get_config(100, 50, "bf16", batched=True)["band"] == 12
        assert binding.get_config(100, 50, "bf16")["band"] == 12
    finally:
        binding.force_config(None)


def test_missing_file_rejected(tmp_path):
    with pytest.raises(binding.ClucsoError):
        binding.load_tuning(str(tmp_path / "nope.json"))


def test_force_overrides_table(tmp_path):
    binding.load_tuning(write(tmp_path, table([entry("split_bf16", 0, 0, 4, "persistent", 8)])))
    binding.force_config(3, "staged", 24, frame=0)
    assert binding.get_config(100, 50, "bf16") == {"products": 3, "schedule": "staged",
                                                    "band": 24, "frame": 0, "source": "forced",
                                                    "bucket": -1}
    assert binding.get_config(100, 50, "fp64")["frame"] == 0
    assert binding.get_config(100, 50, "bf16x4")["products"] == 4
    binding.force_config(None)
    assert binding.get_config(100, 50, "bf16")["source"] == "table"
    with pytest.raises(binding.ClucsoError):
        binding.force_config(5, "staged", 16)
    with pytest.raises(binding.ClucsoError):
        binding.force_config(3, "staged", 0)
    with pytest.raises(binding.ClucsoError):
        binding.force_config(3, "staged", 16, frame=3)


def test_committed_table_covers_every_bucket():
    if not os.path.exists(COMMITTED):
        pytest.skip("no committed tuning table yet")
    t = json.load(open(COMMITTED))
    assert t["arch"] == "gfx950"
    binding.load_tuning(COMMITTED)
    nN, nL = len(t["n_edges"]), len(t["l_edges"])
    seen = {(e["precision"], e["n_bucket"], e["l_bucket"], e.get("call", "single"))
            for e in t["entries"]}
    calls = {e.get("call", "single") for e in t["entries"]}
    for call in calls:
        for prec in ("fp32", "split_bf16", "split_fp16", "split_bf16x4"):
            for i in range(nN):
                for j in range(nL):
                    assert (prec, i, j, call) in seen, (prec, i, j, call)
    # each entry's choice is its fastest measured candidate (within the margin
    # that keeps the default) and what the library reports for the bucket
    name = {"fp32": "fp32", "split_bf16": "bf16", "split_fp16": "fp16", "split_bf16x4": "bf16x4"}
    for e in t["entries"]:
        key = f"x{e['products']}/{e['schedule']}/{e['band']}"
        if "frame" in e:
            key += f"/f{e['frame']}"
        assert key in e["ms"]
        assert e["ms"][key] <= min(e["ms"].values()) * 1.0201
        c = binding.get_config(e["N"], e["L"], name[e["precision"]],
                               batched=e.get("call") == "batched")
        frame = e.get("frame", 1) if e["schedule"] == "staged" else 0
        assert (c["products"], c["schedule"], c["band"], c["frame"], c["source"]) == \
            (e["products"], e["schedule"], e["band"], frame, "table")
    binding.load_tuning(None)


def test_parser_survives_arbitrary_text(tmp_path):
    """Random and truncated inputs: the parser rejects or accepts them but
    never crashes, and a rejected file leaves the loaded table unchanged."""
    hyp = pytest.importorskip("hypothesis")
    st = hyp.strategies
    good = json.dumps(table([entry("split_bf16", 0, 0, 4, "persistent", 8)]))
    binding.load_tuning(write(tmp_path, good, "good.json"))
    before = binding.get_config(100, 50, "bf16")
    path = tmp_path / "fuzz.json"

    @hyp.settings(max_examples=300, deadline=None, derandomize=True)
    @hyp.given(st.one_of(st.text(max_size=200),
                         st.integers(0, len(good)).map(lambda n: good[:n]),
                         st.lists(st.sampled_from(list('{}[]",:0123456789.-e truefalsnul')),
                                  max_size=120).map("".join)))
    def check(text):
        path.write_text(text)
        try:
            binding.load_tuning(str(path))
        except binding.ClucsoError:
            assert binding.get_config(100, 50, "bf16") == before
            return
        binding.load_tuning(write(tmp_path, good, "good.json"))   # accepted: restore

    check()
