"""Train the learned surrogate with the library's own kernels and write a
checkpoint.

The network is trained on transitions of the FP64 integrator (a digester
field of seed 5 run as the coupling driver runs it: feed mask, step,
advection; 174,784 particles x 96 coupling steps, about 2^24 transitions),
96 epochs of Adam with a cosine schedule at batch 8192, particle split
90/5/5 with seed 4, output biases calibrated on half of the validation rows.

    python -m paper_2311_08927_amd.train_surrogate --out PATH

The checkpoint the benchmark's headline comparison loads,
paper_2311_08927_amd/data/surrogate_field.npz, was written by this command.
"""
from __future__ import annotations

import argparse
import sys


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--epochs", type=int, default=96)
    ap.add_argument("--train-steps", type=int, default=96)
    ap.add_argument("--train-seed", type=int, default=4)
    ap.add_argument("--train-data", choices=["field", "batched"], default="field")
    ap.add_argument("--gas-weight", type=float, default=1.0)
    args = ap.parse_args()
    import torch

    from . import adm1 as A
    from . import surrogate as S
    from . import workloads as W
    torch.cuda.set_device(0)
    n_train = W.pad_ld(((1 << 24) + args.train_steps - 1) // args.train_steps, 64)
    ctx = A.Context(n_train, rtol=1e-8, atol=W.atol_vector(1e-8))
    sur = S.Surrogate(ctx, n_train, 8192)
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    rec = S.train_on_transitions(ctx, sur, args.train_data, 1 << 24, args.train_steps,
                                 args.epochs, args.train_seed, args.gas_weight, True, log)
    rec["command"] = "python -m paper_2311_08927_amd.train_surrogate " + " ".join(sys.argv[1:])
    S.save_checkpoint(args.out, sur, rec)
    print(rec)


if __name__ == "__main__":
    main()
