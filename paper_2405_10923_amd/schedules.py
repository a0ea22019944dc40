"""Blocked-schedule choices: (inner panel width, outer panel width, transform
tiles per workgroup of the refresh pass) for rhqr_factor's opts; outer 0 means
one level of panels, tpw 0 lets the library choose from n.

``lookup`` returns the autotuner's entry for the storage type and problem
size bucket when tuned_schedules.json holds one (autotune.py writes it), and
the defaults otherwise: two levels, panels of 8 columns in outer panels of
32, for 8- and 4-byte storage; one level of 16 for 2-byte storage.
"""

DEFAULT = {"float64": (8, 32), "float32": (8, 32), "float16": (16, 0), "bfloat16": (16, 0)}


def dtype_name(dt):
    return str(dt).split(".")[-1]


def default(dt):
    """(panel, outer) for a torch dtype or its name."""
    return DEFAULT[dtype_name(dt)]


def lookup(dt, n, m):
    """(panel, outer, tpw, source) for a factorization of n x m in storage
    type ``dt``: the autotuned entry of its size bucket, or the default."""
    from . import autotune
    name = dtype_name(dt)
    ent = autotune.load().get(autotune.key(name, n, m))
    if ent:
        return ent["panel"], ent["outer"], ent.get("tpw", 0), "autotuned"
    p, o = DEFAULT[name]
    return p, o, 0, "default"
