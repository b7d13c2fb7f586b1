"""Helpers for the GPU tests: fixtures, contexts and the parity criterion."""

import os
import sys

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def load_fixture(idx):
    return dict(np.load(os.path.join(GOLDEN, f"oracle_cfg{idx}.npz")))


def parity_ratios(out, ref, V=None):
    """Per-walker error ratios of the parity criterion (each must be <= tol):
      |d ln|psi||  / max(1, |ln|psi||)
      ||d grad||   / max(1, ||grad||)
      |d lap|      / max(1, |lap| + ||grad||^2)
      |d E_loc|    / max(1, |lap| + ||grad||^2 + |E_loc|)
    The E_loc scale is the size of the cancelling kinetic terms."""
    la, g, lp, el = (np.asarray(out[k]) for k in ("logabs", "grad", "lap", "eloc"))
    rla, rg, rlp, rel = (np.asarray(ref[k]) for k in ("logabs", "grad", "lap", "eloc"))
    B = la.shape[0]
    gn = np.linalg.norm(rg.reshape(B, -1), axis=1)
    kin = np.abs(rlp) + gn**2
    return {
        "logabs": np.abs(la - rla) / np.maximum(1, np.abs(rla)),
        "grad": np.linalg.norm((g - rg).reshape(B, -1), axis=1) / np.maximum(1, gn),
        "lap": np.abs(lp - rlp) / np.maximum(1, kin),
        "eloc": np.abs(el - rel) / np.maximum(1, kin + np.abs(rel)),
    }


def summarize(ratios):
    return {k: (float(np.percentile(v, 50)), float(np.percentile(v, 99)), float(v.max()))
            for k, v in ratios.items()}
