"""Oracle species of every scenario of the 256-scenario mix, computed by the culled
oracle in a pool of worker processes; prints one JSON line per scenario with its
richness and the SHA-256 of its species array (u64, sample order).  Test
infrastructure only: a GPU test runs it as a separate process (which never touches
the GPU, so its workers may fork) and compares the digests with the library's
output.

    python tests/oracle_pool.py [--dw 2.0] [--workers 16]
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)

_WORKLOADS = None


def _culled(k_dw):
    import oracle
    k, dw = k_dw
    w = _WORKLOADS[k]
    osc = oracle.Scenario(w.capacity, w.weights, w.nu, mode=w.mode)
    species, _, _ = osc.simulate_culled(w.seeds[0], w.samples, dw)
    return k, oracle.richness(species), hashlib.sha256(species.astype("<u8").tobytes()).hexdigest()


def main():
    global _WORKLOADS
    ap = argparse.ArgumentParser()
    ap.add_argument("--dw", type=float, default=2.0, help="horizon step of the culled oracle")
    ap.add_argument("--workers", type=int, default=16)
    args = ap.parse_args()
    from paper_2108_05815_amd import workloads as W
    _WORKLOADS = W.config4()
    order = sorted(range(len(_WORKLOADS)), key=lambda k: -len(_WORKLOADS[k].samples))
    n = max(1, min(args.workers, os.cpu_count() or 1))
    with mp.get_context("fork").Pool(processes=n) as pool:
        for k, rich, digest in pool.imap_unordered(_culled, [(k, args.dw) for k in order], chunksize=1):
            print(json.dumps({"k": k, "richness": rich, "sha256": digest}), flush=True)


if __name__ == "__main__":
    main()
