"""Blocked-schedule choices per storage type: (inner panel width, outer panel
width) for rhqr_factor's opts, 0 meaning one level of panels.

The defaults are the fastest measured on a 2^22 x 256 factorization with an
SRHT of l = 1024 on one MI355X: two levels, panels of 8 columns in outer panels
of 32, for 8- and 4-byte storage; one level of 16 for 2-byte storage.
"""

DEFAULT = {"float64": (8, 32), "float32": (8, 32), "float16": (16, 0), "bfloat16": (16, 0)}


def dtype_name(dt):
    return str(dt).split(".")[-1]


def default(dt):
    """(panel, outer) for a torch dtype or its name."""
    return DEFAULT[dtype_name(dt)]
