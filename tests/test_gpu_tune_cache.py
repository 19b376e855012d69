"""The TTM launch-shape table on disk (include/cpqr.h, tune_cache.h).

A first process meets the float32 TTM shapes of a problem, times their launch
shapes and writes the file; a second process with the same file finds every
shape there (nothing is timed again, so the file is left as it was) and, its
launch shapes being the same, reproduces the first run's fits bit for bit.
With CPQR_TUNE_CACHE=off nothing is written.
"""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import json, sys
sys.path[:0] = [sys.argv[1], sys.argv[1] + "/tests"]
import numpy as np
import paper_2503_18759_amd as P
import synthgen as G
P.load_library()
prob = G.make_problem([64, 96, 80], 8, seed=7, rho=0.01, dtype=np.float32)
x, d = P.to_device(prob.X)
r = P.cp_als_qr(x, 8, prob.init, 5, dims=d, tree="restructured")
path, dev = P.tune_cache_path()
print("RESULT " + json.dumps({"fits": [float(f).hex() for f in r["fits"]], "path": path, "device": dev}))
"""


def _run(env_value):
    env = dict(os.environ)
    env["CPQR_TUNE_CACHE"] = env_value
    p = subprocess.run([sys.executable, "-c", SCRIPT, ROOT], env=env, capture_output=True, text=True,
                       timeout=240)
    assert p.returncode == 0, p.stderr[-2000:]
    line = [l for l in p.stdout.splitlines() if l.startswith("RESULT ")][-1]
    return json.loads(line[len("RESULT "):])


def test_tuning_file_is_written_and_reused(tmp_path):
    import paper_2503_18759_amd as P
    path = str(tmp_path / "sub" / "ttm_tune.json")
    a = _run(path)
    assert a["path"] == path and os.path.exists(path)
    text = open(path).read()
    n = P.tune_cache_check(text, a["device"])
    assert n >= 1
    assert P.tune_cache_check(text, a["device"] + "x") == 0
    keys = json.loads(text)["entries"]
    assert all(k.startswith("ttm/p1/") for k in keys)
    assert all(v[0] in (1, 2, 4) and v[1] in (1, 2) for v in keys.values())
    b = _run(path)
    assert open(path).read() == text
    assert b["fits"] == a["fits"]


def test_tuning_file_off(tmp_path):
    c = _run("off")
    assert c["path"] == ""
    assert not any(tmp_path.iterdir())
