"""Command-line driver of Algorithm 1 on one GPU, with checkpoints, a
per-iteration JSONL log and resume.

    python -m paper_2306_03651_amd.run --graph ba --n 100000 --k 50 \\
        --checkpoint ck.json --log it.jsonl --result res.json [--resume]

The run advances one iteration per library call (centra_progressive_
resumable with stop_after = the next iteration, resuming from the previous
call's checkpoint on the same context, which keeps the sample, the
incidence and the AMCERA counts).  After each iteration it appends the
iteration's record to the log, then replaces the checkpoint file.  A run
started with --resume reads the checkpoint, drops log records past it and
continues; the library redraws the sample of the checkpoint's m_i (samples
are functions of their indices), so the result is the uninterrupted run's.

Setting CENTRA_FAULT_AFTER_ITER=i makes the process end abruptly
(os._exit(FAULT_EXIT), no cleanup) right after iteration i is recorded:
a host-forced failure for testing recovery; the device work has finished
by then.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

from . import binding, inputs

FAULT_EXIT = 75
LOG_FIELDS = ["i", "m", "coverage", "sum_topk", "deg_topk", "b_max", "delta_i", "amcera", "wimpy", "xi", "nu",
              "rtilde", "r", "eta", "certified", "ms_sample", "ms_cover", "ms_mcera", "arcs", "nodes"]
RESULT_FIELDS = ["n_picked", "iterations", "certified", "coverage", "m_final", "c_hat", "amcera", "wimpy", "xi",
                 "nu", "rtilde", "r", "eta"]
SCHEDULES = {"geometric": binding.CENTRA_SCHEDULE_GEOMETRIC, "adaptive": binding.CENTRA_SCHEDULE_ADAPTIVE}
SPACES = {"paths": binding.CENTRA_SPACE_SHORTEST_PATHS, "bidir": binding.CENTRA_SPACE_PATHS_BIDIR,
          "triangles": binding.CENTRA_SPACE_TRIANGLES, "kpaths": binding.CENTRA_SPACE_KPATHS}
METHODS = {"centra": binding.CENTRA_METHOD_CENTRA, "hedge": binding.CENTRA_METHOD_HEDGE_P}


def make_graph(a) -> inputs.CSRGraph:
    if a.graph == "ba":
        return inputs.ba_graph(a.n, a.m0, a.graph_seed)
    if a.graph == "grid":
        return inputs.grid_graph(a.side)
    if a.graph == "rmat":
        return inputs.rmat_graph(a.scale, a.edge_factor, seed=a.graph_seed)
    raise SystemExit(f"unknown graph kind {a.graph}")


def make_params(a) -> binding.Params:
    return binding.Params(a.k, a.t, a.eps, a.delta, a.seed, a.instance, a.m_init, a.m_max, a.growth_num,
                          a.growth_den, SCHEDULES[a.schedule], SPACES[a.space], a.kappa, METHODS[a.method])


def record(it) -> dict:
    return {f: (float(getattr(it, f)) if isinstance(getattr(it, f), float) else int(getattr(it, f)))
            for f in LOG_FIELDS}


def write_atomic(path: str, text: str) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write(text)
        f.flush()
        os.fsync(f.fileno())
    os.replace(tmp, path)


def append_line(path: str, obj: dict) -> None:
    with open(path, "a") as f:
        f.write(json.dumps(obj, sort_keys=True) + "\n")
        f.flush()
        os.fsync(f.fileno())


def trim_log(path: str, last_i: int) -> None:
    """Drops log records of iterations after last_i (written after the
    checkpoint that a resume starts from)."""
    if not os.path.exists(path):
        return
    with open(path) as f:
        keep = [line for line in f if line.strip() and json.loads(line)["i"] <= last_i]
    write_atomic(path, "".join(keep))


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--graph", choices=["ba", "grid", "rmat"], default="ba")
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--m0", type=int, default=5)
    ap.add_argument("--side", type=int, default=256)
    ap.add_argument("--scale", type=int, default=16)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--graph-seed", type=int, default=1)
    ap.add_argument("--k", type=int, default=50)
    ap.add_argument("--t", type=int, default=64)
    ap.add_argument("--eps", type=float, default=0.01)
    ap.add_argument("--delta", type=float, default=0.1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--instance", type=int, default=0)
    ap.add_argument("--m-init", type=int, default=100_000)
    ap.add_argument("--m-max", type=int, default=4_000_000)
    ap.add_argument("--growth-num", type=int, default=2)
    ap.add_argument("--growth-den", type=int, default=1)
    ap.add_argument("--schedule", choices=sorted(SCHEDULES), default="geometric")
    ap.add_argument("--space", choices=sorted(SPACES), default="paths")
    ap.add_argument("--kappa", type=int, default=0)
    ap.add_argument("--method", choices=sorted(METHODS), default="centra")
    ap.add_argument("--checkpoint", required=True, help="checkpoint file (JSON), replaced after each iteration")
    ap.add_argument("--log", required=True, help="per-iteration JSONL log")
    ap.add_argument("--result", required=True, help="final result (JSON)")
    ap.add_argument("--resume", action="store_true", help="continue from --checkpoint")
    return ap.parse_args(argv)


def main(argv=None) -> int:
    a = parse(argv)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("run.py needs a HIP device")
    fault_after = int(os.environ.get("CENTRA_FAULT_AFTER_ITER", "0") or 0)
    g = make_graph(a)
    p = make_params(a)
    ctx = binding.centra_create(0, 0)
    dg = binding.DeviceGraph(ctx, g)
    try:
        ck = None
        if a.resume:
            with open(a.checkpoint) as f:
                saved = json.load(f)
            if saved.get("version") != binding.CENTRA_CHECKPOINT_VERSION:
                raise SystemExit("checkpoint version mismatch")
            ck = binding.Checkpoint.from_dict(saved)
            trim_log(a.log, ck.i)
        else:
            for path in (a.log, a.checkpoint, a.result):
                if os.path.exists(path):
                    os.remove(path)
        while True:
            nxt = ck.i + 1 if ck is not None else 1
            rc, picks, res, its, new_ck = binding.centra_progressive_resumable(ctx, dg.handle, p, ck, stop_after=nxt,
                                                                              log_cap=max(nxt, 64))
            for i in sorted(its):
                append_line(a.log, record(its[i]))
            if rc != binding.CENTRA_STOPPED:
                break
            write_atomic(a.checkpoint, json.dumps(new_ck.to_dict(), sort_keys=True) + "\n")
            ck = new_ck
            if fault_after and ck.i == fault_after:
                print(f"fault injected after iteration {ck.i}", flush=True)
                torch.cuda.synchronize()
                os._exit(FAULT_EXIT)
        out = {f: getattr(res, f) for f in RESULT_FIELDS}
        out["picks"] = [int(x) for x in np.asarray(picks, dtype=np.uint32)]
        out["rc"] = int(rc)
        out["graph_hash"] = dg.hash()
        out["params_hash"] = binding.centra_params_hash(p)
        write_atomic(a.result, json.dumps(out, sort_keys=True) + "\n")
        print(json.dumps({"iterations": res.iterations, "certified": res.certified, "m_final": res.m_final,
                          "eta": res.eta}), flush=True)
    finally:
        dg.release()
        binding.centra_destroy(ctx)
    return 0


if __name__ == "__main__":
    sys.exit(main())
