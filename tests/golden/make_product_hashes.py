"""Write SHA-256 digests of the oracle's products at the headline sizes.

Calls only the oracle (oracle/gf2x_oracle.c through oracle.mul) on the seeded
inputs of paper_1708_09746_amd.inputs; nothing comes from the GPU library.
Output: tests/golden/product_sha256.txt, one line per workload:
    <name> <na_bits> <nb_bits> <seed_a> <seed_b> <out_words> <sha256 of the product words, little-endian>
Run:  python tests/golden/make_product_hashes.py [threads]
"""
import hashlib
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1708_09746_amd import inputs  # noqa: E402

WORKLOADS = [
    ("c1", 1 << 16, 1 << 16),
    ("c2", 1 << 20, 1 << 20),
    ("c3a", 1 << 28, 1 << 28),
    ("c3b", 1 << 29, 1 << 29),
]


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count() or 1
    out_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "product_sha256.txt")
    lines = ["# SHA-256 of oracle products (written by make_product_hashes.py; oracle only)",
             "# name na_bits nb_bits seed_a seed_b out_words sha256"]
    for name, na, nb in WORKLOADS:
        sa, sb = inputs.SEEDS[name]
        a = inputs.random_poly(sa, na)
        b = inputs.random_poly(sb, nb)
        t0 = time.time()
        c = oracle.mul(a, na, b, nb, threads=threads)
        dt = time.time() - t0
        digest = hashlib.sha256(c.tobytes()).hexdigest()
        lines.append(f"{name} {na} {nb} {sa:#x} {sb:#x} {len(c)} {digest}")
        print(f"{name}: {dt:.1f} s  {digest}", flush=True)
        with open(out_path, "w") as f:
            f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
