"""Oracle work for the full-size parity tests, run in worker processes (imports the oracle and
NumPy only, never the GPU library)."""
from oracle import sequential


def bdf1_from(job):
    """The oracle's BDF1 step to level n from the given level n-1 (sequential Newton)."""
    p, n, prev = job
    u, _, _ = sequential.bdf1_step(prev, p, n)
    return n, u
