"""Write oracle heights for the benchmark workloads into tests/golden/.

Every stored value comes from the CPU oracle (oracle.fast, pinned by the
oracle tests) run on the seeded inputs of workloads.py; nothing here touches
the HIP library.  Each output is an .npz holding the heights (int8: 1..10, 0 =
infinite), the number of theta applications per surface, and the SHA-256 of
the generated inputs so that a changed generator is detected.

Run:  python tests/golden/make_golden.py [config ...] [--threads N]
"""
import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import fast  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def input_digest(F, P):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(F, dtype=np.uint8).tobytes())
    h.update(np.ascontiguousarray(P, dtype=np.int32).tobytes())
    return h.hexdigest()


def run(name, threads):
    F, P = workloads.CONFIGS[name]()
    n = F.shape[0]
    H = np.zeros(n, dtype=np.int8)
    IT = np.zeros(n, dtype=np.int8)
    t0 = time.time()
    done = [0]

    def one(i):
        h, it = fast.height(F[i], int(P[i]), 10, with_iters=True)
        return i, h, it

    # order the slow primes first so the pool stays busy
    order = sorted(range(n), key=lambda i: -int(P[i]))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for i, h, it in ex.map(one, order):
            H[i], IT[i] = h, it
            done[0] += 1
            if done[0] % 2048 == 0:
                print("%s: %d/%d (%.0f s)" % (name, done[0], n, time.time() - t0), flush=True)
    out = os.path.join(HERE, "heights_%s.npz" % name)
    np.savez_compressed(out, heights=H, theta_iters=IT, sha256=np.array(input_digest(F, P)))
    print("%s: wrote %s in %.0f s" % (name, out, time.time() - t0), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="*", default=list(workloads.CONFIGS))
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    args = ap.parse_args()
    for name in args.configs:
        run(name, args.threads)


if __name__ == "__main__":
    main()
