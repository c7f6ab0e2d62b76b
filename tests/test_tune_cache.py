"""The autotuner cache (l1ls_tune_get / l1ls_tune_set): in-process store and
the JSON file named by L1LS_TUNE_CACHE, read by a later process.  No GPU:
these calls touch no device."""
import json
import os
import subprocess
import sys

import paper_1503_03520_amd as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_set_get_forget():
    assert L.tune_get("test_key/3") == -1
    L.tune_set("test_key/3", 2)
    assert L.tune_get("test_key/3") == 2
    L.tune_set("test_key/3", -1)
    assert L.tune_get("test_key/3") == -1
    assert L.lib().l1ls_tune_set(b'bad"key', 1) == -1
    assert L.lib().l1ls_tune_set(b"", 1) == -1


def test_cache_file_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    env = dict(os.environ, L1LS_TUNE_CACHE=path, L1LS_HIP_MALLOC="1")
    code = ("import sys; sys.path.insert(0, %r); import paper_1503_03520_amd as L; "
            "L.tune_set('fista_f32_residual/27', 3); L.tune_set('batch_rounds/12', 1)") % ROOT
    subprocess.run([sys.executable, "-c", code], env=env, check=True)
    data = json.load(open(path))
    assert data["choices"] == {"batch_rounds/12": 1, "fista_f32_residual/27": 3}
    code = ("import sys; sys.path.insert(0, %r); import paper_1503_03520_amd as L; "
            "print(L.tune_get('fista_f32_residual/27'), L.tune_get('batch_rounds/12'), L.tune_get('x/1'))") % ROOT
    out = subprocess.run([sys.executable, "-c", code], env=env, check=True, capture_output=True, text=True)
    assert out.stdout.split() == ["3", "1", "-1"]
