"""Wide random sweeps of the property tests on the GPU: fresh random draws (not
hypothesis's derandomised ones) for a time budget per sweep, every failure printed with
the case that produced it.

    python -m tests.wide_sweep rollout,mixed,loop,adjoint,batch,pose,frames,voxel,arm,server 60 777

Arguments: the sweeps, seconds per sweep, seed.  Not collected by pytest."""
import contextlib
import io
import os
import sys
import time
import traceback

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import torch  # noqa: E402,F401  (before the library: one HIP runtime)

from paper_2606_12579_amd import gmapp  # noqa: E402
from tests import test_property as tp  # noqa: E402
from tests import test_property_loop as tl  # noqa: E402
from tests import test_property_frames as tf  # noqa: E402
from tests import test_property_batch as tb  # noqa: E402
from tests import test_property_adjoint as ta  # noqa: E402
from tests import test_property_pose_voxel as tpv  # noqa: E402
from tests import test_property_arm as tar  # noqa: E402
from tests import test_property_server as tsv  # noqa: E402


def draw(rng, mode):
    """One case of a sweep, over the ranges of that test's hypothesis strategies."""
    i = lambda a, b: int(rng.integers(a, b + 1))
    b = lambda: bool(rng.integers(0, 2))
    seed = i(0, 2 ** 31 - 1)
    if mode == "rollout":
        return dict(seed=seed, n_o=i(0, 64), n_a=i(1, 8), n_k=i(1, 20), moving=b(), cutoff=i(0, 1), coincide=b(),
                    on_centre=b(), tiling=tp.TILINGS[i(0, len(tp.TILINGS) - 1)])
    if mode == "mixed":
        return dict(seed=seed, n_o=i(0, 64), n_a=i(1, 8), n_k=i(1, 20), moving=b(), cutoff=i(0, 1), coincide=b(),
                    on_centre=b(), tiling=tp.TILINGS[i(0, len(tp.TILINGS) - 1)])
    if mode == "loop":
        return dict(seed=seed, n_o=i(0, 64), n_a=i(1, 8), n_k=i(1, 20), moving=b(), cutoff=i(0, 1), mixed=b(),
                    n_cycles=i(1, 6), ctrl_steps=i(1, 8), ctrl_dt=[0.001, 0.005, 0.01][i(0, 2)],
                    alpha=[0.5, 0.9, 0.99, 1.0][i(0, 3)], t0=float(rng.uniform(0, 0.05)), incumbent=i(-1, 7),
                    tiling=tl.LOOP_TILINGS[i(0, len(tl.LOOP_TILINGS) - 1)])
    if mode == "frames":
        return dict(seed=seed, n_frames=i(0, 3), size=tf.SIZES[i(0, len(tf.SIZES) - 1)],
                    bad_frac=[0.0, 0.05, 0.5, 1.0][i(0, 3)], levels=[0, 20][i(0, 1)],
                    voxel=[0.005, 0.01, 0.05, 0.2][i(0, 3)], min_count=i(1, 3), n_spheres=[-1, 0, 1, 4][i(0, 3)],
                    cap_frac=[0.0, 0.5, 1.0, 2.0][i(0, 3)])
    if mode == "batch":
        jobs = [(i(0, 2 ** 31 - 1), i(0, 200), i(0, 24), i(1, 40), b(), i(0, 1)) for _ in range(i(1, 5))]
        tune = ([0, 64, 96, 256, 4096][i(0, 4)], i(0, 2), [0, 1, 4, 16][i(0, 3)], i(0, 8))
        return dict(jobs=jobs, tune=tune, quantum=[0, 1, 5, 13][i(0, 3)])
    if mode == "adjoint":
        return dict(seed=seed, n_o=i(1, 150), n_a=i(1, 8), n_k=i(2, 60), moving=b(), ckpt=i(1, 64),
                    kf=[0.005, 0.01, 0.02][i(0, 2)])
    if mode == "pose":
        return dict(seed=seed, n_o=i(1, 120), n_a=i(1, 8), n_k=i(2, 40), moving=b(), cutoff=i(0, 1), mixed=b(),
                    tiling=tpv.POSE_TILINGS[i(0, len(tpv.POSE_TILINGS) - 1)])
    if mode == "voxel":
        return dict(seed=seed, n=i(0, 3000), voxel=[0.001, 0.003, 0.01, 0.25][i(0, 3)],
                    lo=tuple(float(np.float32(rng.uniform(-2, 2))) for _ in range(3)),
                    dims=tuple(i(1, 300) for _ in range(3)), min_count=i(1, 3),
                    cap_frac=[0.0, 0.5, 1.0, 2.0][i(0, 3)], static=b())
    if mode == "arm":
        return dict(seed=seed, n_a=i(1, 8), n_o=i(0, 200), n_k=i(2, 40), moving=b(), joints=i(1, 7),
                    damping=[0.0, 0.01, 0.1][i(0, 2)], mixed=b(),
                    tiling=tar.ARM_TILINGS[i(0, len(tar.ARM_TILINGS) - 1)])
    if mode == "server":
        reqs = [(i(0, 2 ** 31 - 1), i(0, 200), i(0, 12), i(1, 60), b(), i(0, 1), b()) for _ in range(i(1, 6))]
        return dict(reqs=reqs, budget=[1 << 20, 64 << 20][i(0, 1)], slots=i(1, 4), quantum=i(1, 32), spread=b())
    raise ValueError(mode)


FN = {"rollout": tp.test_random_tiny_problems, "mixed": tl.test_random_mixed_ensembles,
      "loop": tl.test_random_planning_loops, "frames": tf.test_random_frames_to_voxels,
      "batch": tb.test_random_batches, "adjoint": ta.test_random_adjoint, "pose": tpv.test_random_pose_problems,
      "voxel": tpv.test_random_voxel_passes, "arm": tar.test_random_arm_problems,
      "server": tsv.test_random_request_mixes}


def main():
    modes = sys.argv[1].split(",")
    budget = float(sys.argv[2])
    seed = int(sys.argv[3])
    ctx = gmapp.Context(0)
    fails = 0
    for mode in modes:
        rng = np.random.default_rng([seed, sorted(FN).index(mode)])
        fn = FN[mode].hypothesis.inner_test
        t0, n, mf = time.time(), 0, 0
        while time.time() - t0 < budget:
            kw = draw(rng, mode)
            buf = io.StringIO()
            try:
                with contextlib.redirect_stdout(buf):
                    fn(ctx, **kw)
            except AssertionError:
                fails += 1
                mf += 1
                print(f"FAIL [{mode} #{n}] {kw}", flush=True)
                if mf <= 6:
                    print(buf.getvalue()[-2000:])
                    traceback.print_exc(limit=3)
                    sys.stdout.flush()
            finally:
                ctx.clear_tiling()
            n += 1
            if n % 3000 == 0:
                print(f"  {mode}: {n} cases, {mf} failures", flush=True)
        print(f"== {mode}: {n} cases, {mf} failures in {time.time() - t0:.0f} s", flush=True)
    ctx.close()
    print(f"== failures {fails}", flush=True)
    return 1 if fails else 0


if __name__ == "__main__":
    sys.exit(main())
