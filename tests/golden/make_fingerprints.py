"""Writes tests/golden/fingerprints.txt: SHA-256 fingerprints of the seeded
generator's CSR arrays for the plain workloads and a few batch members.
Calls only the input generator (no oracle values, no GPU path)."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402


def main():
    lines = ["# name n nnz sha256 (written by make_fingerprints.py)"]
    for i in (1, 2, 3):
        m = synth.config(i)
        lines.append(f"config{i} {m.n} {m.nnz} {synth.fingerprint(m)}")
    for k in (0, 1, 2, 3, 4095):
        m = synth.batch_member(k)
        lines.append(f"batch{k} {m.n} {m.nnz} {synth.fingerprint(m)}")
    with open(os.path.join(HERE, "fingerprints.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
