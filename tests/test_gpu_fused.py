"""GPU test of the product fused with the next step's first TSQR level.

For n_next in {2, 4} and a next unfolding of n_next r <= 32 columns (W with
m <= 8 columns up to 8, m <= 32 beyond), the decomposition builds each row
tile of the next unfolding Y = reshape(W V) (Sec. 4.1.2) in registers,
stores it and runs the flat Householder reduction of Sec. 3.2 on the same
registers.  The product accumulates in the order of the TSMM kernel and the
reduction is the rows or cooperative body itself, so the result must
equal, bit for bit, the decomposition with separate launches, which a child
process computes with TTSVD_TSMM_QR=0 on the same input (the switch is read
once per process).  Shapes: n = 2 (the first steps of a QTT: 2 x 2 -> 4,
4 x 4 -> 8, 8 x 8 -> 16, 16 x 16 -> 32 columns) and n = 4 (4 x 2 -> 8,
4 x 4 -> 16, 16 x 8 -> 32), in FP64, FP32 and BF16 storage, with r < KB
(3 of 4 columns per block) once; the inputs span many row tiles and slices
and end in ragged tiles.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2102_00104_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU host
    pytest.skip("no GPU", allow_module_level=True)

import paper_2102_00104_amd as tt  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CASES = [([2] * 21, 8, "f64"), ([2] * 20 + [3], 6, "f32"), ([2] * 21, 8, "bf16"),
         ([4] * 10, 2, "f64"), ([2] * 22, 16, "f64"), ([2] * 21, 16, "f32"),
         ([4] * 9, 4, "f64"), ([4] * 9, 8, "bf16")]
TORCH_DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}

CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
import paper_2102_00104_amd as tt
from paper_2102_00104_amd import synth
dims = [int(x) for x in sys.argv[2].split(',')]
X = synth.uniform(dims, seed=int(sys.argv[3]))
dt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[sys.argv[5]]
Xd = torch.from_numpy(X).to("cuda:0").to(dt)
g = tt.ttsvd_decompose(Xd, dims, int(sys.argv[4]), 0.0)
np.savez(sys.argv[6], ranks=np.array(g.ranks), sig=np.concatenate([np.asarray(s, dtype=np.float64) for s in g.sigma[1:]]),
         *[c.cpu().numpy() for c in g.cores])
"""


def decompose(dims, r_max, name, seed):
    X = synth.uniform(dims, seed=seed)
    Xd = torch.from_numpy(X).to(torch.device("cuda:0")).to(TORCH_DT[name])
    return tt.ttsvd_decompose(Xd, dims, r_max, 0.0)


@pytest.mark.parametrize("dims,r_max,name", CASES)
def test_fused_equals_separate_launches(dims, r_max, name, tmp_path):
    seed = 61 + len(dims)
    # the fused kernel runs (event profile of this process)
    tt.ttsvd_profile_reset()
    tt.ttsvd_profile_enable(True)
    try:
        g = decompose(dims, r_max, name, seed)
        torch.cuda.synchronize()
        names = [k["name"] for k in tt.ttsvd_profile_read()]
    finally:
        tt.ttsvd_profile_enable(False)
        tt.ttsvd_profile_reset()
    assert any(n.startswith("tsmm_qr") for n in names), names
    out = str(tmp_path / "separate.npz")
    env = dict(os.environ, TTSVD_TSMM_QR="0")
    print("child: separate launches for", dims, r_max, name, flush=True)
    subprocess.run([sys.executable, "-c", CHILD, ROOT, ",".join(map(str, dims)), str(seed),
                    str(r_max), name, out], env=env, check=True, timeout=240)
    ref = np.load(out)
    assert list(ref["ranks"]) == list(g.ranks)
    sig = np.concatenate([np.asarray(s, dtype=np.float64) for s in g.sigma[1:]])
    assert np.array_equal(ref["sig"], sig)
    for i, c in enumerate(g.cores):
        assert np.array_equal(ref["arr_%d" % i], c.cpu().numpy()), "core %d" % (i + 1)
