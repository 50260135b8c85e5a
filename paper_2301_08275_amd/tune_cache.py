"""Write the launch-shape tuning cache (gpe_autotune per shape class).

Run on the target GPU:

    python -m paper_2301_08275_amd.tune_cache OUT.json

It times the candidate launch shapes of every shape class listed below (the
benchmark grids and the serving mix's classes, both precisions) and saves the
table as JSON.  Callers load it with gpe_tuning_load before creating contexts
or a server; bench.py loads the copy shipped beside this file.
"""
import os
import sys
import time

# (shape, precision): the 2D/3D workload grids and the serving mix's classes
PRECS = ("fp64", "fp32", "fp32s")
CLASSES = [((n, n, n), p) for n in (512, 256, 128, 64) for p in PRECS]
CLASSES += [((1024, 1024, 1024), p) for p in PRECS]
CLASSES += [((n, n), p) for n in (512, 256, 128, 64) for p in PRECS]

SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_mi355x.json")


def main(out):
    import torch

    torch.cuda.set_device(0)
    from paper_2301_08275_amd import gpe

    gpe.gpe_tuning_clear()
    for shape, prec in CLASSES:
        t0 = time.time()
        d = gpe.make_desc(shape, 0.0, 1.0, 1.0, prec)
        sites = 1
        for n in shape:
            sites *= n
        steps = 6 if sites >= 1 << 30 else 24 if sites >= 1 << 24 else 64
        t = gpe.gpe_autotune(d, steps=steps)
        print("%-16s %s %s (%.1f s)" % ("x".join(map(str, shape)), prec, t, time.time() - t0),
              flush=True)
    gpe.gpe_tuning_save(out)
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else SHIPPED)
