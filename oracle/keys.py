"""CPU oracle of the single stages measured on their own (test infrastructure only; only the
test suite uses it).  Plain definitions, no blocking or reordering.

sort_keys (Section V-C): the ascending order of the keys, duplicates kept -- what every
LSD pass sequence over the key's digits, each pass stable, produces.

merge_runs (Section IV-C): the merge of two ascending runs, taking keys one at a time from
the front of either run, the smaller first and run A's on equal keys.
"""

import numpy as np


def sort_keys(keys: np.ndarray) -> np.ndarray:
    """Ascending order of an unsigned integer array (a library sort as the one step)."""
    return np.sort(np.asarray(keys), kind="stable")


def merge_runs(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """The two-finger merge of ascending runs a and b (a's key first on ties)."""
    a = np.asarray(a)
    b = np.asarray(b)
    out = np.empty(a.size + b.size, dtype=np.result_type(a, b))
    # b[t] lands after every key of a that is <= it and after b's t earlier keys
    pos = np.searchsorted(a, b, side="right") + np.arange(b.size)
    mask = np.zeros(out.size, dtype=bool)
    mask[pos] = True
    out[mask] = b
    out[~mask] = a
    return out
