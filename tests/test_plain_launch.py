"""The persistent kernels launched without the cooperative flag (RSK_COOPERATIVE=0, read once per
process, so those solves run in a child process; the cooperative ones run in the test's own
process, which holds the device's cooperative-launch resources once it has made such a launch):
the same grid, hence the same iteration, bit for bit, for the register-tile and general dense
kernels, the CSR grid kernel and a batched launch."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2203_10838_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_SOLVES = r'''
import numpy as np
import torch
from paper_2203_10838_amd import inputs, rsk
dev = torch.device("cuda:0")
T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
out = {}
d = inputs.dense_system(3000, 2048, 60, seed=91)
idx = inputs.index_stream(inputs.row_sampling_weights(d["A"]), 40, 300, 92)
for kern in (1, 2):
    r = rsk.solve_dense(T(d["A"]), T(d["b"]), lam=0.3, eta=300, alpha=40.0, K=40, index_stream=T(idx), kernel=kern)
    out[f"dense{kern}"] = r.x_star.cpu().numpy()
c = inputs.csr_system(20000, 5000, 16, 40, seed=93)
ic = inputs.index_stream(inputs.csr_sampling_weights(c["row_ptr"], c["val"]), 50, 64, 94)
r = rsk.solve_csr(T(c["row_ptr"]), T(c["col"]), T(c["val"]), 5000, T(c["b"]), lam=0.2, eta=64, alpha=20.0, K=50,
                  index_stream=T(ic), kernel=2)
out["csr"] = r.x_star.cpu().numpy()
sys_ = []
for i in range(3):
    s = inputs.dense_system(800 + 300 * i, 200 + 100 * i, 10, seed=95 + i)
    e = 1 + (200 + 100 * i) // 10
    sys_.append(rsk.BatchSystem(A=T(s["A"]), b=T(s["b"]), index_stream=T(inputs.index_stream(
        inputs.row_sampling_weights(s["A"]), 30, e, 98 + i)), eta=e, K=30, alpha=float(e), lam=0.2))
rb = rsk.solve_batched(sys_)
for i in range(3):
    out[f"batched{i}"] = rb.x_star[i].cpu().numpy()
'''

_CHILD = "import sys\nsys.path.insert(0, sys.argv[1])\n" + _SOLVES + "np.savez(sys.argv[2], **out)\n"


def _plain(tmp_path):
    f = str(tmp_path / "out_plain.npz")
    env = dict(os.environ, RSK_COOPERATIVE="0")
    print("child solve, RSK_COOPERATIVE=0", flush=True)
    res = subprocess.run([sys.executable, "-c", _CHILD, ROOT, f], env=env, capture_output=True, text=True,
                         timeout=240)
    assert res.returncode == 0, res.stderr[-2000:]
    return dict(np.load(f))


def _cooperative():
    assert os.environ.get("RSK_COOPERATIVE", "1") != "0", "the test process must launch cooperatively"
    scope = {}
    exec(_SOLVES, scope)
    return scope["out"]


def test_plain_launch_equals_cooperative(rsk_lib, cuda, tmp_path):
    coop = _cooperative()
    plain = _plain(tmp_path)
    assert sorted(plain) == sorted(coop)
    for k in coop:
        assert np.array_equal(plain[k], coop[k]), k
        assert np.isfinite(coop[k]).all() and np.abs(coop[k]).max() > 0, k
