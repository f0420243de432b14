"""Writes tests/golden/c1_seed<S>_paper.txt: the oracle's partition structure of the C1
matrix (4096^2, seed S) under [VDIA, VBR(literal search), CSR] with delta 0.75 / 0.5 and
A_min 256 / 256. Calls only oracle/ (the literal block search takes minutes on the CPU,
which is why its result is stored).

    python tests/golden/make_c1_paper.py 0
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2407_00829_amd.synth import gen_c1  # noqa: E402


def main(seed: int) -> None:
    A, _ = gen_c1(seed)
    th = oracle.Thresholds(amin_band=256, amin_block=256)
    P = oracle.plan(A, [oracle.VDIA, oracle.VBR, oracle.CSR], oracle.MODE_PAPER, th)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"c1_seed{seed}_paper.txt")
    with open(out, "w") as f:
        f.write(f"# Oracle partition of gen_c1({seed}) (4096x4096, nnz {A.nnz}) under [VDIA, VBR "
                "literal search, CSR], delta 0.75 / 0.5, A_min 256 / 256; written by "
                "tests/golden/make_c1_paper.py\n")
        f.write("seg_row_start " + " ".join(map(str, P["seg_row_start"].tolist())) + "\n")
        f.write("seg_nrows " + " ".join(map(str, P["seg_nrows"].tolist())) + "\n")
        f.write("idiag " + " ".join(map(str, P["idiag"].tolist())) + "\n")
        f.write("blk " + " ".join(map(str, P["blk"].ravel().tolist())) + "\n")
        f.write(f"csr_nnz {P['csr_col'].size}\n")
    print(out)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 0)
