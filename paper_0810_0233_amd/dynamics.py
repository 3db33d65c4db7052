"""A caller-side time step for repeated evaluation as the moments evolve.

The method computes the field H of given moments; a simulation then moves the
moments and asks again, on the same geometry, so one plan (and its captured
evaluation) serves every step.  The step here is plain precession of unit
moments about the local field, m <- normalise(m + dt m x H), written with
torch on the device buffers in place (the captured evaluation reads the same
addresses).  It is the application around the method, not part of it.
"""


def precession_step_(d_m, d_H, dt):
    """In-place explicit precession step of unit moments d_m [B][n][3] (FP64
    device tensor) in the field d_H of the same shape."""
    import torch

    d_m.add_(torch.linalg.cross(d_m, d_H, dim=-1), alpha=dt)
    d_m.div_(torch.linalg.vector_norm(d_m, dim=-1, keepdim=True))
    return d_m
