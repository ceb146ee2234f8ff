"""The sweep's two addressing forms give identical results.

Where the rows of a level are whole 64-column tiles, a wavefront covers one
row segment and its north / south rows are wave-uniform offsets; the sweep
kernel can then address the buffers from the lowest row involved with the row
offsets in scalar registers (by default only the FP32 prolongation sweep does,
TPMG_SWEEP_ROWS=1 makes every sweep that can, 0 none).  Only the addresses
differ, so the outputs must agree bit for bit: the sweeps (zero guess,
general, with prolongation) on every level and the V-cycle are computed in
child processes under each setting and compared.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from gpu_util import device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, {root!r})
import paper_1605_00492_amd as tp
n, nz, levels = 256, 13, 3
rng = np.random.default_rng(1605)
c = 1.0 + 0.5 * rng.random((3, nz, n, n))
dz = [1.05 ** k for k in range(nz)]
dev = torch.device("cuda:0")
out = {{}}
for prec in ("fp64", "mixed"):
    H = tp.Hierarchy(torch.from_numpy(c).to(dev), dz=dz, a_h=4.0, a_z=1e4, levels=levels, precision=prec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    vec = lambda l: torch.from_numpy(rng.standard_normal((nz, n >> l, n >> l))).to(dev, dt)
    for l in range(levels):
        b, u = vec(l), vec(l)
        out[f"{{prec}}_zero_{{l}}"] = H.smooth(b, level=l)
        out[f"{{prec}}_general_{{l}}"] = H.smooth(b, u, level=l)
        if l + 1 < levels:
            out[f"{{prec}}_prolong_{{l}}"] = H.prolong_smooth(u, vec(l + 1), b, level=l)
    out[f"{{prec}}_vcycle"] = H.vcycle(vec(0))
    torch.cuda.synchronize()
    H.close()
np.savez({path!r}, **{{k: v.cpu().numpy() for k, v in out.items()}})
print("child ok", flush=True)
"""


def _run(tmp_path, setting):
    path = str(tmp_path / f"rows_{setting}.npz")
    env = dict(os.environ)
    env.pop("TPMG_SWEEP_ROWS", None)
    if setting != "default":
        env["TPMG_SWEEP_ROWS"] = setting
    print(f"[gpu] sweep rows child TPMG_SWEEP_ROWS={setting}", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, path=path)], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    with np.load(path) as f:
        return {k: f[k] for k in f.files}


def test_row_addressing_matches_generic(tmp_path):
    device()
    ref = _run(tmp_path, "0")
    for setting in ("default", "1"):
        got = _run(tmp_path, setting)
        assert sorted(got) == sorted(ref)
        diff = [k for k in ref if not np.array_equal(got[k], ref[k])]
        print(f"[gpu] TPMG_SWEEP_ROWS={setting}: {len(ref)} outputs, differing {json.dumps(diff)}", flush=True)
        assert not diff, diff
