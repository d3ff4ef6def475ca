"""Autotuner: pick the fastest kernel variant per database shape and batch size.

Every variant (tile shape, LDS pipeline depth, rows per wave) computes the
same exact product; they differ only in speed, which depends on the
database shape and the batch size (the paper likewise picks its tile sizes
from the query count and dimensions, Algorithm 4).  The tuner times each
valid variant with HIP events on the device and records the fastest in a
JSON table keyed by ``"RxC"`` and batch size; :func:`apply` installs a
table entry on an open database with ``pir_db_set_variant``.  Row-gathered
products (the incremental hint after a refresh) are timed apart, on a
random 1% of the rows, and recorded under ``"r<n>"``: scattered rows favour
deeper pipelines than the whole database does.

    python -m paper_2510_03631_amd.tune --shape 32768x32768 --batches 0,64,1024 \
        --rows-batches 1024 --out paper_2510_03631_amd/tiles.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys

from ._lib import Database, PirError, variant_names

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles.json")


def _time_call(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / reps * 1e3   # microseconds


def tune_database(db: Database, batches, reps: int = 5, log=print, modulus: int = 0,
                  rows_frac: float = 0.0) -> dict:
    """Time every valid variant for each batch size; return {batch: {name: us}}.

    With ``modulus`` set, batched calls are timed in the field form
    (``answer_batch_modp``), which runs only the split-K capable variants.
    With ``rows_frac`` set, each batch size ``n`` is timed as the incremental
    hint over that fraction of the rows (``hint_update_rows``) and keyed
    ``"r<n>"``.
    """
    import torch
    results = {}
    for B in batches:
        names = variant_names(B)
        gathered = rows_frac > 0 and B > 0
        if gathered:
            m = max(1, round(rows_frac * db.rows))
            rows = torch.randperm(db.rows, device=db.device)[:m].to(torch.int32)
            A = torch.randint(-2**31, 2**31 - 1, (db.cols, B), dtype=torch.int32, device=db.device)
            H = torch.zeros((db.rows, B), dtype=torch.int32, device=db.device)
            ws = db.workspace(B)
            # The refresh as the library runs it: A's limb planes prepared
            # once, each call timing the gathered product alone.
            planes = db.hint_planes(A)
            fn = lambda: db.hint_update_rows_planes(rows, planes, B, H, ws=ws)
        elif B == 0:
            q = torch.randint(-2**31, 2**31 - 1, (db.cols,), dtype=torch.int32, device=db.device)
            out = torch.empty(db.rows, dtype=torch.int32, device=db.device)
            ws = db.workspace(0)
            fn = lambda: db.answer(q, out=out, ws=ws)
        else:
            Q = torch.randint(-2**31, 2**31 - 1, (db.cols, B), dtype=torch.int32, device=db.device)
            out = torch.empty((db.rows, B), dtype=torch.int32, device=db.device)
            ws = db.workspace(B)
            if modulus:
                fn = lambda: db.answer_batch_modp(Q, modulus, out=out, ws=ws)
            else:
                fn = lambda: db.answer_batch(Q, out=out, ws=ws)
        times = {}
        key = f"r{B}" if gathered else B
        for v, name in enumerate(names):
            if v == 0 or (modulus and B and not name.startswith(("ring", "narrow", "few"))):
                continue
            try:
                db.set_variant(B, v, rows=gathered)
            except PirError:
                continue   # not valid for this database / batch
            times[name] = _time_call(fn, reps)
            log(f"  {db.rows}x{db.cols} B={key!s:>6} {name:18s} {times[name]:10.1f} us")
        db.set_variant(B, 0, rows=gathered)
        results[key] = times
    return results


def best(results: dict) -> dict:
    return {str(B): min(t, key=t.get) for B, t in results.items() if t}


def load(path: str = DEFAULT_TABLE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def apply(db: Database, table: dict = None) -> int:
    """Install the table's choices for this database's shape; returns how many."""
    table = load() if table is None else table
    entry = table.get(f"{db.rows}x{db.cols}", {})
    n = 0
    for B, name in entry.get("best", {}).items():
        gathered = B.startswith("r")
        try:
            db.set_variant(int(B[1:] if gathered else B), name, rows=gathered)
            n += 1
        except (PirError, ValueError):
            pass
    return n


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--shape", action="append", required=True, help="RxC, repeatable")
    ap.add_argument("--batches", default="0,1,8,32,64,128,256,1024")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--modulus", type=int, default=0,
                    help="time the field form mod this prime (Goldberg shapes)")
    ap.add_argument("--rows-batches", default="",
                    help="hint widths n to time as incremental hints (row-gathered)")
    ap.add_argument("--rows-frac", type=float, default=0.01,
                    help="fraction of the rows an incremental hint recomputes")
    args = ap.parse_args(argv)
    import torch
    import workload
    table = load(args.out)
    batches = [int(b) for b in args.batches.split(",") if b]
    rows_batches = [int(b) for b in args.rows_batches.split(",") if b]
    for shp in args.shape:
        R, C = (int(x) for x in shp.lower().split("x"))
        D = workload.device_db(R, C, workload.SEED_BASE + 77, "cuda")
        with Database(D) as db:
            log = lambda m: print(m, flush=True)
            res = tune_database(db, batches, args.reps, log=log, modulus=args.modulus)
            if rows_batches:
                res.update(tune_database(db, rows_batches, args.reps, log=log,
                                         rows_frac=args.rows_frac))
        entry = table.setdefault(f"{R}x{C}", {"best": {}, "us": {}})
        entry["best"].update(best(res))          # merge: other batch sizes keep their choice
        entry["us"].update({str(B): t for B, t in res.items()})
        del D
        torch.cuda.empty_cache()
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(f"wrote {args.out}")
    return 0


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    sys.exit(main())
