"""Autotune the stored-band pentadiagonal solvers over a grid of (length, batch) shapes.

    python -m paper_1806_10550_amd.tune [--out FILE] [--lengths 128,256,...] [--batches 16,256,...]

Each shape is timed by tf_autotune for plain and for transposed solves (partitioned,
Thomas with 64/128/256 lines per workgroup, block cyclic reduction for lengths <= 2048)
and appended as one JSON line to
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
    a = ap.parse_args(argv)
    import torch

    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    out = a.out or os.path.join(HERE, f"autotune_{arch}.jsonl")
    if os.path.exists(out):
        os.remove(out)
    for t in (False, True):
        for n in [int(x) for x in a.lengths.split(",")]:
            for b in [int(x) for x in a.batches.split(",")]:
                if n * b > a.max_cells:
                    continue
                choice = lib.autotune(n, b, out, transposed=t)
                print(f"{'transposed' if t else 'plain':10s} length {n:6d} batch {b:6d}: {choice}", flush=True)
    print(out)


if __name__ == "__main__":
    main()
