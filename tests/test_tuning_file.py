"""The autotuner's JSON file (xeng_tuning_save / xeng_tuning_load), on the
host: these calls touch no device. A file round-trips through the process
cache entry for entry, a file that does not parse changes nothing, and the
allocation-free entry point rejects what it cannot run before any device
call."""
import ctypes
import json

import pytest

from paper_1411_3751_amd import xeng

GOOD = {
    "format": "xeng-tuning", "version": 1,
    "subarrays": [
        {"arch": "gfx950", "n_inputs": 64, "n_chans": 512, "n_time": 4096, "in_bits": 4,
         "engine": 0, "kernel": "small_n", "tile": 64},
        {"arch": "gfx950", "n_inputs": 300, "n_chans": 8, "n_time": 1000, "in_bits": 8,
         "engine": 0, "kernel": "register_staging", "tile": 64},
        {"arch": "gfx942", "n_inputs": 512, "n_chans": 128, "n_time": 8192, "in_bits": 4,
         "engine": 0, "kernel": "persistent_workgroup", "tile": 128},
    ],
    "batches": [
        {"arch": "gfx950", "shapes": [[64, 512, 4096, 4, 0], [256, 256, 4096, 4, 0]],
         "kernels": [["small_n", 64], ["persistent_workgroup", 128]],
         "workgroups_per_cu": 2, "order": 1},
    ],
}


def entries(doc):
    subs = {json.dumps(e, sort_keys=True) for e in doc["subarrays"]}
    bats = {json.dumps(e, sort_keys=True) for e in doc["batches"]}
    return subs, bats


def test_round_trip(tmp_path):
    src, dst = tmp_path / "in.json", tmp_path / "out.json"
    src.write_text(json.dumps(GOOD))
    xeng.tuning_clear()
    assert xeng.tuning_load(str(src)) == 4
    assert xeng.tuning_save(str(dst)) == 4
    out = json.loads(dst.read_text())
    assert out["format"] == "xeng-tuning" and out["version"] == 1
    assert entries(out) == entries(GOOD)
    # loading merges: the same file again changes nothing
    assert xeng.tuning_load(str(dst)) == 4
    assert xeng.tuning_save(str(dst)) == 4
    assert entries(json.loads(dst.read_text())) == entries(GOOD)
    xeng.tuning_clear()
    assert xeng.tuning_save(str(dst)) == 0
    assert json.loads(dst.read_text()) == {"format": "xeng-tuning", "version": 1,
                                           "subarrays": [], "batches": []}


def bad_docs():
    yield "not json", "{"
    yield "wrong format", json.dumps({"format": "other", "version": 1})
    yield "wrong version", json.dumps({"format": "xeng-tuning", "version": 2})
    d = json.loads(json.dumps(GOOD))
    d["subarrays"][0]["kernel"] = "no_such_kernel"
    yield "unknown kernel", json.dumps(d)
    d = json.loads(json.dumps(GOOD))
    d["subarrays"][1]["tile"] = 48
    yield "bad register tile", json.dumps(d)
    d = json.loads(json.dumps(GOOD))
    d["batches"][0]["kernels"].pop()
    yield "kernels and shapes differ", json.dumps(d)
    d = json.loads(json.dumps(GOOD))
    d["batches"][0]["workgroups_per_cu"] = 0
    yield "bad schedule", json.dumps(d)
    d = json.loads(json.dumps(GOOD))
    d["subarrays"][0]["n_inputs"] = 6.5
    yield "non-integer shape", json.dumps(d)


@pytest.mark.parametrize("name,text", list(bad_docs()), ids=[n for n, _ in bad_docs()])
def test_malformed_files_change_nothing(tmp_path, name, text):
    f, out = tmp_path / "bad.json", tmp_path / "out.json"
    f.write_text(text)
    xeng.tuning_clear()
    with pytest.raises(xeng.XengError) as e:
        xeng.tuning_load(str(f))
    assert "bad.json" in str(e.value)
    assert xeng.tuning_save(str(out)) == 0


def test_missing_and_unwritable_paths(tmp_path):
    with pytest.raises(xeng.XengError):
        xeng.tuning_load(str(tmp_path / "absent.json"))
    with pytest.raises(xeng.XengError):
        xeng.tuning_save(str(tmp_path / "no_dir" / "out.json"))
    lib = xeng.load()
    assert lib.xeng_tuning_load(None, None) == xeng.XENG_EINVAL
    assert lib.xeng_tuning_save(None, None) == xeng.XENG_EINVAL


def static_call(sub, samples=0x1000, out=0x2000):
    lib = xeng.load()
    s = xeng.Subarray(*sub)
    return lib.xeng_correlate_dump_static(ctypes.byref(s), ctypes.c_void_p(samples),
                                          ctypes.c_void_p(out), None)


@pytest.mark.parametrize("sub,words", [
    ((100, 4, 64, 4, 0), "multiple of 16"),         # not the persistent kernel's shape
    ((512, 4, 40000, 4, 0), "at most 32768"),       # more than one segment
    ((512, 4, 0, 4, 0), "n_time"),                  # bad shape
    ((4096, 1000, 64, 4, 0), "tiles"),              # tile list beyond the static array
])
def test_static_entry_point_rejects_before_any_device_call(sub, words):
    assert static_call(sub) == xeng.XENG_EINVAL
    assert words in xeng.load().xeng_last_error().decode()


def test_static_entry_point_rejects_null_and_misaligned_pointers():
    assert static_call((512, 4, 64, 4, 0), samples=0) == xeng.XENG_EINVAL
    assert static_call((512, 4, 64, 4, 0), samples=0x1001) == xeng.XENG_EINVAL
    assert "aligned" in xeng.load().xeng_last_error().decode()
    assert static_call((512, 4, 64, 4, 0), out=0x2004) == xeng.XENG_EINVAL
    assert "aligned" in xeng.load().xeng_last_error().decode()
