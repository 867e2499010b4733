"""Write tests/golden/knn_model_test.txt using the CPU oracle only.

Small matrices from the four workload families (2D Laplacian, 3D
variable-coefficient diffusion, band of half-width 8, Erdos-Renyi graph
Laplacian) are labelled the way the paper labels its sample: Algorithm I is
run for every eps1 = 10^-t, t = 2..7, and the class is the t with the smallest
I = omega * N1 + N2 (eq. 4), ties to the larger eps1.  Features are the
oracle's (n, m, 2BFS pseudo-diameter, v over the first 20 FP32 iterations).

omega = 0.6 is the ratio of FP32 to FP64 bytes moved per CG iteration for
these matrix shapes (about 0.58-0.62), the right order for a bandwidth-bound
GPU.  The model only has to be a fixed, oracle-made input for the parity tests.

    python tests/golden/make_test_model.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OMEGA = 0.6


def features_and_label(a, b):
    dummy = oracle.KnnModel.from_samples(np.array([[1.0, 1, 1, 1]]), [2], k=1)
    r = oracle.solve(a, b, oracle.EPS1_AUTO, 1e-10, model=dummy)
    chi = [a.n, a.nnz, r.ell, r.v]
    n1s, n2s = [], []
    for e in oracle.cost.EPS1_CANDIDATES:
        s = oracle.solve(a, b, e, 1e-10)
        n1s.append(s.n1)
        n2s.append(s.n2)
    return chi, oracle.cost.label_from_sweep(n1s, n2s, OMEGA)


def main(out=os.path.join(HERE, "knn_model_test.txt")):
    rng = np.random.default_rng(2024)
    feats, labels = [], []
    for i in range(48):
        fam = W.FAMILIES[i % 4]
        n_target = int(np.exp(rng.uniform(np.log(300), np.log(6000))))
        a = W.family_matrix(fam, n_target, seed=1000 + i)
        _, b = W.rhs(a, seed=1000 + i)
        chi, t = features_and_label(a, b)
        feats.append(chi)
        labels.append(t)
    m = oracle.KnnModel.from_samples(np.array(feats, dtype=np.float64), labels, k=3, mask=15,
                                     omega=OMEGA)
    oracle.save_model(m, out)
    print(f"wrote {out}: {m.ns} samples, classes {np.bincount(m.label, minlength=8)[2:]}")


if __name__ == "__main__":
    main()
