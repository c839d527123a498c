"""The P-bit prefix table of sorted K-bit codes, from its definition: entry p of table j
counts the codes of table j below p << (K - P).  Tests compare an index's exported table
with this table over the oracle's sorted codes, for any prefix width the index chose, and
check that every 2^(P - 13)-th entry is the oracle's own 13-bit table."""
import numpy as np


def prefix_table(tcode: np.ndarray, K: int, P: int) -> np.ndarray:
    bounds = np.arange((1 << P) + 1, dtype=np.uint64) << np.uint64(K - P)
    return np.stack([np.searchsorted(t.astype(np.uint64), bounds, side="left") for t in tcode]).astype(np.uint32)


def check_offsets(got: np.ndarray, o, P: int) -> int:
    """Mismatches of an exported P-bit table against the oracle index o (its codes and its
    own min(13, K)-bit table)."""
    F = o.off.shape[1] - 1
    step = (got.shape[1] - 1) // F
    assert got.shape[1] == (1 << P) + 1 and step * F == (1 << P)
    bad = int(np.count_nonzero(got[:, ::step] != o.off))
    if step > 1:
        bad += int(np.count_nonzero(got != prefix_table(o.tcode, o.K, P)))
    return bad
