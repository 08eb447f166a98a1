"""Accuracy of the learned rollout (precision study), through the C ABI.

For each scene: a network rollout in bf16 and in FP32 operands, against the FP32 mass-spring
simulator over the same simulated time (stride simulator steps per network frame). At every
checkpoint frame, the position RMS (divided by the cloth width), the energy and the maximum
structural stretch are FP64 reductions on the GPU (cloth_reduce_fp64). The simulator reference
itself is held to the FP64 CPU reference by the GPU tests.

    python -m paper_2403_12820_amd.evaluate --scenes 2 --size 256 --checkpoints 1,10,100

Scenes (--scene): "random" (random pins and wind, as in training); "blown" (four corners pinned,
a uniform pressure from below, eq. 3); "ball" (no pins, no wind, dropped onto a ball under its
middle, with the sphere in the constraint of eq. 5). Pressure and ball act in the simulator and as
known terms in the network frames; the network never saw them in training.
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

from . import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))


def make_scenes(kind, size, n_scenes, seed, pressure=20.0, ball=0.3, gap=0.05, friction=0.5):
    """Scenes and their batch for an evaluation kind (see the module notes)."""
    if kind == "random":
        scenes = I.random_scenes([(size, size)] * n_scenes, seed=seed)
        return scenes, I.make_batch(scenes)
    pins = {"blown": "four_corners", "ball": "none"}[kind]
    scenes = [I.make_scene(size, size, pins, seed=seed * 1000003 + b) for b in range(n_scenes)]
    batch = I.make_batch(scenes)
    if kind == "blown":
        batch.pressure = np.full(batch.n, pressure, np.float32)
    else:
        side = (size - 1) * float(batch.h[0])
        batch.sphere = np.array([[side / 2, side / 2, -ball - gap, ball, friction]] * batch.n, np.float32)
    return scenes, batch


def evaluate(theta, size=256, n_scenes=2, checkpoints=(1, 2, 5, 10, 20, 50, 100), stride=10, seed=5, ch=32,
             device="cuda", scene="random", **scene_args):
    import torch
    from . import _lib as L
    mat = I.Material()
    scenes, batch = make_scenes(scene, size, n_scenes, seed, **scene_args)
    plan = L.Plan.from_batch(batch, device)
    sim = L.ms_params(mat)
    s0 = torch.tensor(batch.state, device=device)
    th = torch.tensor(np.asarray(theta, np.float32), device=device)
    red = torch.zeros(4 * batch.n, dtype=torch.float64, device=device)
    width = (batch.W - 1) * batch.h
    nodes = batch.H * batch.W
    e_ref = nodes * batch.mass * 9.8 * width  # energy scale: the cloth's weight over its width

    def reduce(state, ref):
        L.cloth_reduce_fp64(plan, sim, state, ref, red)
        torch.cuda.synchronize()
        return red.cpu().numpy().reshape(-1, 4)

    e0 = reduce(s0, None)[:, 1]
    guard = L.Guard()
    guard.stretch_max, guard.energy_gain_max, guard.check_every, guard.substeps = 1e9, 1e30, 0, stride
    runs = {"bf16": L.PECNN_BF16, "fp32": L.PECNN_FP32}
    models = {k: L.make_model(th, ch, p, dt=stride * mat.dt) for k, p in runs.items()}
    state = {k: [s0.clone(), s0.clone()] for k in runs}
    fb = torch.zeros(batch.n, dtype=torch.int32, device=device)
    ref = [s0.clone(), torch.empty_like(s0)]
    curve = {k: [] for k in list(runs) + ["ms_fp32", "bf16_vs_fp32"]}
    done = 0
    for cp in sorted(set(int(c) for c in checkpoints)):
        n = cp - done
        L.cloth_ms_step(plan, sim, ref[0], ref[1], n * stride)
        ref.reverse()
        for k in runs:
            L.pecnn_rollout(plan, models[k], sim, guard, state[k][0], state[k][1], n, fb, None)
        done = cp
        for k in runs:
            r = reduce(state[k][1], ref[0])
            curve[k].append({"frame": cp, "rms_width": (np.sqrt(r[:, 0] / nodes) / width).tolist(),
                             "energy_drift": ((r[:, 1] - e0) / e_ref).tolist(),
                             "max_structural_stretch": r[:, 2].tolist()})
        r = reduce(ref[0], None)
        curve["ms_fp32"].append({"frame": cp, "energy_drift": ((r[:, 1] - e0) / e_ref).tolist(),
                                 "max_structural_stretch": r[:, 2].tolist()})
        r = reduce(state["bf16"][1], state["fp32"][1])
        curve["bf16_vs_fp32"].append({"frame": cp, "rms_width": (np.sqrt(r[:, 0] / nodes) / width).tolist()})
    return {"scene": scene, **scene_args, "scenes": n_scenes, "grid": size, "stride": stride, "seed": seed,
            "pins": [sc.pin_kind for sc in scenes], "curve": curve}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--weights", default=os.path.join(HERE, "weights", "pecnn_ch32.npy"))
    ap.add_argument("--scenes", type=int, default=2)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--stride", type=int, default=10)
    ap.add_argument("--checkpoints", default="1,2,5,10,20,50,100")
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--scene", choices=("random", "blown", "ball"), default="random")
    ap.add_argument("--pressure", type=float, default=20.0, help="blown: pressure from below, N/m^2")
    ap.add_argument("--ball", type=float, default=0.3, help="ball: radius, m")
    ap.add_argument("--gap", type=float, default=0.05, help="ball: gap below the flat cloth, m")
    ap.add_argument("--friction", type=float, default=0.5, help="ball: friction in [0, 1]")
    args = ap.parse_args()
    theta = np.load(args.weights, allow_pickle=False)
    cps = [int(x) for x in args.checkpoints.split(",")]
    extra = {"blown": {"pressure": args.pressure},
             "ball": {"ball": args.ball, "gap": args.gap, "friction": args.friction}}.get(args.scene, {})
    print(json.dumps(evaluate(theta, args.size, args.scenes, cps, args.stride, args.seed, scene=args.scene, **extra)))


if __name__ == "__main__":
    main()
