"""Write the golden FFT-length table from the oracle (run: python tests/golden/make_golden.py)."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fftlen  # noqa: E402

CASES = [(16, 100), (16, 5000), (64, 1 << 12), (64, 1 << 16), (300, 20000), (1024, 1 << 16),
         (1024, 1 << 20), (4096, 1 << 20), (8192, 1 << 20), (8192, 1 << 22), (8192, 100000),
         (8192, 1 << 14)]

if __name__ == "__main__":
    with open(os.path.join(HERE, "fft_length_rule.txt"), "w") as fh:
        fh.write("# n_c longest n_f  -- FFT length by the halving rule of the Weighting section\n")
        for nc, longest in CASES:
            fh.write(f"{nc} {longest} {fftlen.paper_fft_length(nc, longest)}\n")
