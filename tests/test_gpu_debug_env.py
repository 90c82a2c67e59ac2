"""Debugging switches read from the environment (PCF_SYNC, PCF_TRACE): each
case runs in a child process, since the library reads them once."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import numpy as np, torch
from paper_2405_07122_amd import pcfsort as P, datagen
P.load()
x = datagen.f64("uniform", 300000, 3)
if BAD:
    x[17] = np.nan
d = torch.from_numpy(x).to("cuda")
st = torch.zeros(1, dtype=torch.int32, device="cuda")
try:
    out = P.pcf_sort_f64(d, d_status=st)
    torch.cuda.synchronize()
    rc = 0
    if not BAD:
        assert torch.equal(out, torch.sort(d)[0])
except P.PcfError as e:
    rc = e.code
torch.cuda.synchronize()
print("RC", rc, "STATUS", int(st.cpu()[0]), flush=True)
'''


def _run(bad: bool, env_extra: dict):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    env = dict(os.environ)
    for k in ("PCF_SYNC", "PCF_TRACE"):
        env.pop(k, None)
    env.update(env_extra)
    print(f"[gpu-test] child: bad={bad} env={env_extra}", flush=True)
    r = subprocess.run([sys.executable, "-c", f"BAD = {bad}\n" + CHILD], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [l for l in r.stdout.splitlines() if l.startswith("RC ")][-1].split()
    return int(line[1]), int(line[3]), r.stderr


def test_status_word_call_returns_after_enqueue_by_default():
    from paper_2405_07122_amd import pcfsort as P
    rc, st, _ = _run(True, {})
    assert rc == 0 and st == P.ERR_INVALID_KEY


def test_pcf_sync_returns_the_data_status():
    from paper_2405_07122_amd import pcfsort as P
    rc, st, _ = _run(True, {"PCF_SYNC": "1"})
    assert rc == P.ERR_INVALID_KEY and st == P.ERR_INVALID_KEY
    rc, st, _ = _run(False, {"PCF_SYNC": "1"})
    assert rc == 0 and st == 0


def test_pcf_trace_prints_one_line_per_call():
    rc, st, err = _run(False, {"PCF_TRACE": "1"})
    assert rc == 0 and st == 0
    lines = [l for l in err.splitlines() if l.startswith("pcf: ")]
    assert len(lines) == 1, err[-2000:]
    ln = lines[0]
    assert "f64 n=300000 segments=1 payload=0" in ln and "status=0 overflow=0" in ln
    levels = ln[ln.index("levels=[") + 8:ln.index("]")].split()
    assert levels, ln
    nodes, units, keys = (int(v) for v in levels[0].split("/"))
    assert nodes == 1 and units >= 1 and keys == 300000
