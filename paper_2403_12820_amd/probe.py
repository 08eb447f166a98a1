"""Fixed launches of one kernel of the library on the benchmark workload, for profiler runs.

  python -m paper_2403_12820_amd.probe cnn   # bf16 CNN frame, 128 cloths of 256 x 256, Ch = 32
  python -m paper_2403_12820_amd.probe ms    # FP32 mass-spring step on the same batch
  python -m paper_2403_12820_amd.probe reduce  # FP64 diagnostics (the rollout guard's check)
  python -m paper_2403_12820_amd.probe copy  # plain device copy of 1 GiB (counter calibration)
"""
import sys


def main(kind: str, reps: int = 5, instances: int = 128, size: int = 256):
    import torch
    from paper_2403_12820_amd import _lib as L
    from paper_2403_12820_amd import inputs as I

    dev = torch.device("cuda:0")
    if kind == "copy":
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(reps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copy bytes per launch read %d written %d" % (src.numel() * 4, dst.numel() * 4))
        return
    mat = I.Material()
    batch = I.make_batch(I.random_scenes([(size, size)] * instances, seed=5))
    plan = L.Plan.from_batch(batch, dev)
    s0 = torch.tensor(batch.state, device=dev)
    bufs = [s0.clone(), s0.clone(), torch.empty_like(s0)]
    if kind == "cnn":
        theta = torch.tensor(I.init_theta(32, seed=1), device=dev)
        model = L.make_model(theta, 32, L.PECNN_BF16, dt=10 * mat.dt)
        for i in range(reps):
            L.pecnn_forward(plan, model, bufs[i % 3], bufs[(i + 1) % 3], bufs[(i + 2) % 3])
    elif kind == "ms":
        sim = L.ms_params(mat)
        for i in range(reps):
            L.cloth_ms_step(plan, sim, bufs[i % 2], bufs[(i + 1) % 2], 1)
    elif kind == "reduce":
        sim = L.ms_params(mat)
        out = torch.empty(4 * batch.n, dtype=torch.float64, device=dev)
        for i in range(reps):
            L.cloth_reduce_fp64(plan, sim, bufs[0], bufs[1], out)
    else:
        raise SystemExit("unknown probe " + kind)
    torch.cuda.synchronize()
    print("%s: %d launches over %d nodes" % (kind, reps, batch.total))


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 5)
