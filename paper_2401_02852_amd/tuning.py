"""Autotune cache: the sweep tile shape chosen per (device, n, cost type),
kept as JSON so that a later process can skip the timing runs.

    shapes = tuning.autotune(ctx, [24, 28, 30])        # times, keeps, returns
    tuning.save("tune.json", ctx, shapes)
    tuning.load("tune.json", ctx)                        # applies what matches
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Tuple

from ._binding import Context


def device_key(ctx: Context) -> str:
    import torch
    props = torch.cuda.get_device_properties(ctx.device)
    return f"{props.name}|{getattr(props, 'gcnArchName', '')}|{props.multi_processor_count}"


def autotune(ctx: Context, ns: Iterable[int], cost_dtypes=("u8",), reps: int = 3) -> Dict[Tuple[int, str], dict]:
    out = {}
    for n in ns:
        for dt in cost_dtypes:
            shape = ctx.autotune(n, dt, reps)
            if shape:
                out[(int(n), dt)] = shape
    return out


def save(path: str, ctx: Context, shapes: Dict[Tuple[int, str], dict]) -> None:
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    dev = data.setdefault(device_key(ctx), {})
    for (n, dt), shape in shapes.items():
        dev[f"{n}/{dt}"] = shape
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def load(path: str, ctx: Context) -> int:
    """Applies the saved shapes for this context's device; returns how many."""
    with open(path) as f:
        data = json.load(f)
    count = 0
    for key, shape in data.get(device_key(ctx), {}).items():
        n, dt = key.split("/")
        ctx.set_tune(int(n), shape, dt)
        count += 1
    return count
