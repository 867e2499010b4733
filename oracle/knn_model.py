"""Reader/writer for the kNN model text file (oracle side; test infrastructure).

File layout (one token group per line, '#' starts a comment line):

    mpcg-knn-model 1
    k <int>
    mask <int>            bit j set = feature j of (n, m, ell, v) is used
    omega <float>         t_sp / t_dp used when the labels were made
    ns <int>
    fmin <f> <f> <f> <f>  per-feature minimum over the training sample
    fmax <f> <f> <f> <f>  per-feature maximum over the training sample
    <n> <m> <ell> <v> <t> one training sample per line, t = class 2..7

Floats are written with 17 significant digits so that every reader recovers
the same doubles.
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class KnnModel:
    k: int
    mask: int
    omega: float
    feat: np.ndarray   # (ns, 4) raw features
    label: np.ndarray  # (ns,) int32 classes 2..7
    fmin: np.ndarray   # (4,)
    fmax: np.ndarray   # (4,)

    @property
    def ns(self) -> int:
        return int(self.feat.shape[0])

    @staticmethod
    def from_samples(feat, label, k: int = 5, mask: int = 15, omega: float = 1.0 / 3.0) -> "KnnModel":
        feat = np.asarray(feat, dtype=np.float64).reshape(-1, 4)
        return KnnModel(k=int(k), mask=int(mask), omega=float(omega), feat=feat,
                        label=np.asarray(label, dtype=np.int32),
                        fmin=feat.min(axis=0), fmax=feat.max(axis=0))


def save_model(m: KnnModel, path: str) -> None:
    with open(path, "w") as f:
        f.write("mpcg-knn-model 1\n")
        f.write(f"k {m.k}\nmask {m.mask}\nomega {m.omega:.17g}\nns {m.ns}\n")
        f.write("fmin " + " ".join(f"{v:.17g}" for v in m.fmin) + "\n")
        f.write("fmax " + " ".join(f"{v:.17g}" for v in m.fmax) + "\n")
        for row, t in zip(m.feat, m.label):
            f.write(" ".join(f"{v:.17g}" for v in row) + f" {int(t)}\n")


def load_model(path: str) -> KnnModel:
    lines = [ln.strip() for ln in open(path) if ln.strip() and not ln.lstrip().startswith("#")]
    if not lines or lines[0].split() != ["mpcg-knn-model", "1"]:
        raise ValueError(f"{path}: not an mpcg-knn-model v1 file")
    hdr = {}
    i = 1
    while i < len(lines) and lines[i].split()[0] in ("k", "mask", "omega", "ns", "fmin", "fmax"):
        tok = lines[i].split()
        hdr[tok[0]] = tok[1:]
        i += 1
    ns = int(hdr["ns"][0])
    rows = [ln.split() for ln in lines[i:i + ns]]
    if len(rows) != ns or any(len(r) != 5 for r in rows):
        raise ValueError(f"{path}: expected {ns} sample lines of 5 fields")
    feat = np.array([[float(v) for v in r[:4]] for r in rows], dtype=np.float64).reshape(-1, 4)
    label = np.array([int(r[4]) for r in rows], dtype=np.int32)
    return KnnModel(k=int(hdr["k"][0]), mask=int(hdr["mask"][0]), omega=float(hdr["omega"][0]),
                    feat=feat, label=label,
                    fmin=np.array([float(v) for v in hdr["fmin"]], dtype=np.float64),
                    fmax=np.array([float(v) for v in hdr["fmax"]], dtype=np.float64))
