"""The five workloads: sizes, method parameters and seeds.

c1  plain method, 64^2, 90 angles x 91 rays, 1 angle/block, r=5, lambda=1e-2
c2  plain method, 1024^2, 720 angles x 1449 rays, 8 angles/block, r=10, lambda=1e-3
c3  c1 with bf16-stored image shadow and sinogram
c4  512 slices of 512^2 sharing A, 360 x 725, 4 angles/block, r=8
c4m mixed batch 64 x 256^2, 32 x 512^2, 8 x 1024^2 (360 angles each)
c5  warm start, 256^2, 180 x 363, 1 angle/block, r=5, lambda=1e-2
c3d 3D parallel beam from random directions (the paper's 3D experiment):
    511^3 volume, 1000 directions uniform on the sphere, 511 x 511 detector,
    1 direction/block, r=0, alpha=1 in unit-voxel scaling (lambda = h^2 with
    h = 2/511), 0.1% noise, one epoch
"""
from __future__ import annotations

CONFIGS = {
    "c1": dict(N=64, n_angles=90, g=1, r=5, lam=1e-2, epochs=20, noise=0.01,
               n_ellipses=10, phantom_seed=1001, noise_seed=2001, schedule_seed=3001),
    "c2": dict(N=1024, n_angles=720, g=8, r=10, lam=1e-3, epochs=10, noise=0.01,
               n_ellipses=20, phantom_seed=1002, noise_seed=2002, schedule_seed=3002),
    "c3": dict(N=64, n_angles=90, g=1, r=5, lam=1e-2, epochs=20, noise=0.01,
               n_ellipses=10, phantom_seed=1001, noise_seed=2001, schedule_seed=3001,
               precision="bf16"),
    "c4": dict(N=512, n_slices=512, n_angles=360, g=4, r=8, lam=1e-3, epochs=5,
               noise=0.005, n_ellipsoids=20, phantom_seed=1004, noise_seed=2004,
               schedule_seed=3004),
    "c4m": dict(groups=[(256, 64), (512, 32), (1024, 8)], n_angles=360, g=4, r=8,
                lam=1e-3, epochs=5, noise=0.005, n_ellipsoids=20, phantom_seed=1004,
                noise_seed=2004, schedule_seed=3004),
    "c3d": dict(N=511, n_dirs=1000, n_det=511, g=1, r=0, lam=(2.0 / 511) ** 2, epochs=1,
                noise=0.001, n_ellipsoids=10, phantom_seed=1006, dir_seed=1007,
                noise_seed=2006, schedule_seed=3006),
    "c5": dict(N=256, n_angles=180, g=1, r=5, lam=1e-2, epochs=20, noise=0.01,
               n_ellipses=10, schedule_seed=3005, train_seeds=(10000, 20000),
               test_seeds=(20000, 21000)),
}


def get_config(name: str) -> dict:
    return dict(CONFIGS[name])


def warmstart_sample(seed: int):
    """One sample of the warm-start workload: (x_true[256,256], b[180,363])
    float64; phantom seed ``seed``, noise seed ``seed + 1_000_000``."""
    from .phantom import make_slice_problem
    c = CONFIGS["c5"]
    x, b, _ = make_slice_problem(c["N"], c["n_angles"], c["n_ellipses"], c["noise"], seed,
                                 seed + 1_000_000)
    return x, b
