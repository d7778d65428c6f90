"""slim_project_noalloc: the forward projection through the library's fixed
scratch, for callers that cannot allocate device memory.

Each call is checked against slim_project on the same context (the same
launches, so bit for bit) and against the FP64 oracle (rel. <= 1e-6, the bar
of the forward projector's parity tests), on two calls in a row, the second
with a smaller input, then on a second, smaller context that shares the
device's scratch.  A call that needs more scratch than the array holds is
refused before any launch.
"""
import numpy as np
import pytest

import synth
from oracle import system

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu
pytestmark = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")

if torch.cuda.is_available():
    from paper_1912_07962_amd import Slim, slim


def _rel(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _check_call(s, P, ids, x):
    """project_noalloc into a NaN-filled buffer == project == oracle."""
    ref_gpu = s.project(ids, x)
    got = torch.full_like(ref_gpu, float("nan"))
    s.project_noalloc(ids, x, got)
    torch.cuda.synchronize()
    assert torch.equal(got, ref_gpu)
    xs = x.cpu().numpy().astype(np.float64).reshape(s.B, -1)
    g = got.cpu().numpy().reshape(s.B, len(ids), P.R)
    for k in range(s.B):
        ref = P.forward(ids, xs[k]).reshape(len(ids), P.R)
        assert _rel(g[k], ref) < 1e-6, k


@gpu
def test_noalloc_projection_matches_project_and_oracle():
    N, na, B = 256, 180, 3
    P = system.Projector(N, na)
    xs = np.stack([synth.rasterize(synth.random_ellipses(8, 40 + k), N) for k in range(B)])
    x = torch.as_tensor(xs, dtype=torch.float32, device="cuda")
    s = Slim(N, na, n_slices=B, r=0, lam=1.0)
    # 45 angles of both orientations: several band groups and ray chunks
    _check_call(s, P, list(range(0, 180, 4)), x)
    # a smaller call: the scratch keeps the first call's partial sums, which
    # the second must not read
    _check_call(s, P, [7, 91, 133], x)
    s.close()
    # a second, smaller context on the same device shares the scratch
    N2, na2 = 37, 16
    P2 = system.Projector(N2, na2)
    x2 = torch.as_tensor(synth.rasterize(synth.random_ellipses(5, 9), N2)[None],
                         dtype=torch.float32, device="cuda")
    s2 = Slim(N2, na2, r=0, lam=1.0)
    _check_call(s2, P2, list(range(16)), x2)
    s2.close()


@gpu
def test_noalloc_projection_refuses_more_than_the_scratch():
    # 12 slices x 256 angles x 1449 rays = 4.45 M floats > 4,194,304 whatever
    # the number of band groups
    N, na, B = 1024, 720, 12
    s = Slim(N, na, n_slices=B, r=0, lam=1.0)
    x = torch.zeros((B, N, N), dtype=torch.float32, device="cuda")
    out = torch.full((B, 256, s.R), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(slim.SlimError) as ei:
        s.project_noalloc(list(range(256)), x, out)
    assert ei.value.status == slim.SLIM_EINVAL
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    s.close()
