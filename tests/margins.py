"""Relative-error checks that also report the measured error.

check(label, err, bar) asserts err < bar and prints one line "MARGIN label err bar" (visible
with pytest -s); with the environment variable PIC_MARGINS set to a file path the line is
appended there too, so a run's measured margins can be read back after it ends.
"""
import os


def rel_max(a, b, scale):
    """max |a - b| / scale (scale > 0)."""
    import numpy as np
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / scale)


def check(label, err, bar):
    line = "MARGIN %s %.3e %.1e" % (label, err, bar)
    print(line, flush=True)
    path = os.environ.get("PIC_MARGINS")
    if path:
        with open(path, "a") as f:
            f.write(line + "\n")
    assert err < bar, line
