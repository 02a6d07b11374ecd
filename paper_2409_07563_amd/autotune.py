"""Cache of autotuned launch shapes (see mppi_autotune in include/mppi.h).

A choice is keyed by what decides it: the device architecture, the dynamics,
integrator and cost, the number of samples rounded up to a power of two, the
horizon, the MLP width, the number of batch instances, the cost's synthetic
load (nested cosines) and gradient mode (which has its own launch shapes).  The cache is a
JSON object {key: {"tuning": {...}, "timings": [...]}} written atomically.
"""
from __future__ import annotations

import json
import os
import tempfile


def k_bucket(K: int) -> int:
    b = 1
    while b < K:
        b *= 2
    return b


def arch(device) -> str:
    import torch
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def key(ctl, arch_name: str | None = None) -> str:
    pb = ctl.problems[0]
    hidden = int(getattr(pb, "mlp_hidden", 0) or 0) if pb.model == "bicycle_mlp" else 0
    Ks = [int(q.K) for q in ctl.problems]
    Ts = [int(q.T) for q in ctl.problems]
    return "|".join([arch_name or arch(ctl.device), pb.model, pb.integrator, pb.cost,
                     f"K{k_bucket(max(Ks))}", f"T{max(Ts)}", f"H{hidden}",
                     f"n{ctl.n_inst}", f"sumKT{k_bucket(sum(k * t for k, t in zip(Ks, Ts)))}",
                     f"cos{int(getattr(pb, 'cost_cosines', 0))}",
                     f"grad{int(bool(getattr(ctl, 'requires_grad', False)))}"])


def parse_report(text: str) -> list:
    out = []
    for ln in text.strip().splitlines():
        parts = ln.split()
        if len(parts) < 6:
            continue
        rec = {"phase": parts[0], "us": float(parts[-1])}
        for kv in parts[1:-1]:
            k, v = kv.split("=")
            rec[k] = int(v)
        out.append(rec)
    return out


def load(path: str) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def store(path: str, k: str, result: dict) -> None:
    data = load(path)
    data[k] = {"tuning": result["tuning"], "timings": result.get("timings", [])}
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".autotune")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
