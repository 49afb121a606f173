"""Error measure of the FP32 comparisons: the larger of the relative L2
error and the element max-abs error relative to the largest reference
entry.  The L2 norm alone would let one wrong row (an edge or corner row at
1% of its own amplitude, say) pass under an array-wide 1e-5 bar; the
max-abs term catches any entry off by more than the bar times the array's
scale."""
import numpy as np


def err32(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb, mb = np.linalg.norm(b), np.max(np.abs(b))
    return max(np.linalg.norm(a - b) / max(nb, 1e-300), np.max(np.abs(a - b)) / max(mb, 1e-300))
