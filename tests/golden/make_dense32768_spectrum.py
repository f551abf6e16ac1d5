"""Write dense32768_seed1004_spectrum.txt: the 64 smallest positive
eigenvalues of H for the dense mixed-precision workload (n = 32768,
K = Q1 diag(k) Q1^T, M = Q2 diag(m) Q2^T, Haar Q1, Q2, k, m ~ U[0.5, 10],
seed 1004).

Only the seeded generator and the oracle's closed form run here: the factors
come from gen.dense_factors_torch on the CPU (the draws of gen.dense_factors,
QR by torch), the eigenvalues from oracle.exact.dense_spectrum_smallest_torch
(square roots of the smallest eigenvalues of F^T F, F = diag(sqrt k) Q1^T Q2
diag(sqrt m); Lemma 2.1).
The GPU tests read the file, because the closed form costs about
2.5e14 flops at this size (tens of minutes on a few host cores).

Usage:  python tests/golden/make_dense32768_spectrum.py   (about 40 GiB of RAM)
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

N, SEED, COUNT = 32768, 1004, 64
OUT = os.path.join(HERE, "dense32768_seed1004_spectrum.txt")


def main():
    import gen
    from oracle import exact

    t0 = time.time()
    q1, k, q2, m = gen.dense_factors_torch(N, SEED, "cpu")
    print(f"factors in {time.time() - t0:.0f}s", flush=True)
    lam = exact.dense_spectrum_smallest_torch(q1, k, q2, m, COUNT)
    del q1, q2
    print(f"spectrum in {time.time() - t0:.0f}s", flush=True)
    with open(OUT, "w") as fh:
        fh.write(f"# The {COUNT} smallest positive eigenvalues of H = [[0, K], [M, 0]] for the dense\n"
                 f"# workload K = Q1 diag(k) Q1^T, M = Q2 diag(m) Q2^T, n = {N}, seed {SEED}\n"
                 f"# (gen.dense_factors_torch), from oracle.exact.dense_spectrum_smallest_torch; written by\n"
                 f"# make_dense32768_spectrum.py.  Relative error of the closed form below 1e-13.\n"
                 f"# max k = {k.max():.17g}, max m = {m.max():.17g} (||H||_2 = the larger)\n"
                 f"# columns: index  lambda\n")
        for i, v in enumerate(lam, 1):
            fh.write(f"{i} {v:.17g}\n")
    print(OUT)


if __name__ == "__main__":
    main()
