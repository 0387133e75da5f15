"""Helpers shared by the GPU tests (checks only; no method arithmetic)."""

import numpy as np


def sin_angle(Va, Vb) -> float:
    """Largest principal-angle sine between span(Va) and span(Vb)."""
    Qa, _ = np.linalg.qr(np.asarray(Va))
    Qb, _ = np.linalg.qr(np.asarray(Vb))
    return float(np.linalg.norm(Qb - Qa @ (Qa.conj().T @ Qb), 2))


def banner(msg: str) -> None:
    print(f"[gpu] {msg}", flush=True)


def to_np(t):
    return t.detach().cpu().numpy()
