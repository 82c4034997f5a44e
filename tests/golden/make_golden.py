"""Write the stored expected values under tests/golden/ that are not printed
in the paper.  Calls only the CPU oracle.

    python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402


def main():
    c1, c2 = O.comb_tables(32)
    with open(os.path.join(HERE, "comb_tables_c32.txt"), "w") as f:
        f.write("# Default combination arrays of the neighbour-exchange variant (group size 32),\n")
        f.write("# written by tests/golden/make_golden.py from the oracle's Fisher-Yates draw.\n")
        f.write("comb1 = " + " ".join(str(int(v)) for v in c1) + "\n")
        f.write("comb2 = " + " ".join(str(int(v)) for v in c2) + "\n")
    arr = O.bbs_comb_tables(32)
    with open(os.path.join(HERE, "bbs_comb_tables_c32.txt"), "w") as f:
        f.write("# Default arrangement arrays of the BBS-based variant (Algorithm 5, group size 32),\n")
        f.write("# written by tests/golden/make_golden.py from the oracle's Fisher-Yates draw.\n")
        for a in range(16):
            f.write(f"array{a} = " + " ".join(str(int(v)) for v in arr[a]) + "\n")


if __name__ == "__main__":
    main()
