"""Autotune the stored-band pentadiagonal solvers and the forward x sweep over a grid of
(length, batch) shapes.

    python -m paper_1806_10550_amd.tune [--out FILE] [--lengths 128,256,...] [--batches 16,256,...]
                                        [--xs-lengths ...] [--xs-batches ...]

Each shape is timed by tf_autotune for plain and for transposed solves (partitioned,
Thomas with 64/128/256 lines per workgroup, block cyclic reduction for lengths <= 2048),
and each x-sweep shape (row length, number of rows) by tf_autotune_xsweep (partitioned
against whole-row), and appended as one JSON line to
FILE (default: autotune_<arch>.jsonl beside this module). tf_autotune_load (or
lib.autotune_load) reads the file back; entries of other GPU architectures are skipped.
"""
import argparse
import os

from . import lib

HERE = os.path.dirname(os.path.abspath(__file__))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out")
    ap.add_argument("--lengths", default="128,256,512,1024,2048,4096,8192")
    ap.add_argument("--batches", default="16,256,512,4096,65536")
    ap.add_argument("--max-cells", type=int, default=1 << 27, help="skip shapes with more cells")
    ap.add_argument("--xs-lengths", default="64,128,256,384,512,768,1024,1536,2048,3072,4096,8192")
    ap.add_argument("--xs-batches", default="64,256,1024,2048,4096,8192")
    ap.add_argument("--only", choices=["all", "solvers", "xsweep"], default="all",
                    help="solvers / xsweep: re-tune one kind and keep the other kind's lines of FILE")
    a = ap.parse_args(argv)
    import torch

    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    out = a.out or os.path.join(HERE, f"autotune_{arch}.jsonl")
    keep = []
    if os.path.exists(out):
        if a.only != "all":
            with open(out) as f:
                keep = [ln for ln in f if ('"kind": "xsweep"' in ln) == (a.only == "solvers")]
        os.remove(out)
    with open(out, "w") as f:
        f.writelines(keep)
    for t in ((False, True) if a.only != "xsweep" else ()):
        for n in [int(x) for x in a.lengths.split(",")]:
            for b in [int(x) for x in a.batches.split(",")]:
                if n * b > a.max_cells:
                    continue
                choice = lib.autotune(n, b, out, transposed=t)
                print(f"{'transposed' if t else 'plain':10s} length {n:6d} batch {b:6d}: {choice}", flush=True)
    for n in ([int(x) for x in a.xs_lengths.split(",")] if a.only != "solvers" else []):
        for b in [int(x) for x in a.xs_batches.split(",")]:
            if n * b > a.max_cells:
                continue
            choice = lib.autotune_xsweep(n, b, out)
            print(f"x sweep    length {n:6d} rows  {b:6d}: {choice}", flush=True)
    print(out)


if __name__ == "__main__":
    main()
