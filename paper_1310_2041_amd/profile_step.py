"""Short fused-step run used as the target of rocprofv3 counter passes.

python -m paper_1310_2041_amd.profile_step [--config c3|c4] [--steps 12] [--halo 2] [--brick 0 (auto)] [--sort-every 30]

c1..c3: the workload's start, the first half step and `steps` fused steps
(reporting energies every step) in the benchmark's configuration (deposit
halo, sort interval, fused pass with the density deposit).
c4: the 64-replica A10B10 sweep stepped `steps` times through the batched
entry points (sorting every 10, energies on the last step).
Both end with a plain 1 GiB device copy whose FETCH_SIZE / WRITE_SIZE
readings calibrate the counters (bytes per reported KiB).
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_BYTES = 1 << 30


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c3")
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--halo", type=int, default=2)
    ap.add_argument("--brick", type=int, default=0)
    ap.add_argument("--sort-every", type=int, default=30)
    args = ap.parse_args()
    import torch

    from paper_1310_2041_amd import engine
    from synth import workloads as wl

    if args.config == "c4":
        systems = [wl.build_replica(sp, r) for r, sp in enumerate(wl.replica_specs())]
        b = engine.BatchState(systems, sort_every=10)
        del systems
        b.start()
        b.step(args.steps, report_last=True)
    else:
        s = wl.build(wl.SPECS[args.config])
        st = engine.HpfState.from_system(s, halo=args.halo, sort_brick=args.brick)
        del s
        st.start(sort=True)
        st.prime()
        for k in range(args.steps):
            st.step_fused(report=True, sort=k % args.sort_every == 0)
    torch.cuda.synchronize()
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print("profile_step done", flush=True)


if __name__ == "__main__":
    main()
