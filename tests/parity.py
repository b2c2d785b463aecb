"""Element-by-element comparison of GPU outputs with the oracle's."""
import numpy as np


def mismatches(got, want):
    bad = []
    for key in ("flags", "counts", "label"):
        if not np.array_equal(np.asarray(got[key]), np.asarray(want[key])):
            bad.append(key)
    for grp in ("parts", "local", "contigs"):
        for key, val in want[grp].items():
            if key == "status":
                continue
            g = got[grp].get(key)
            if isinstance(val, np.ndarray):
                if g is None or g.shape != val.shape or not np.array_equal(g, val):
                    bad.append("%s.%s" % (grp, key))
            elif g != val:
                bad.append("%s.%s (%r != %r)" % (grp, key, g, val))
    return bad
