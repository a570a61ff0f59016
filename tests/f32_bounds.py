"""Error bounds of the FP32 offset form against the FP64 oracle (shared by
the GPU tests of the single-tree and batched FP32 forms)."""
import numpy as np

RHO_F32 = 1e-6   # relative, per vertex
POPULATED = 64   # particles whose leaf touches a vertex, for the plain relative bound


def check_rho_f32(o, x, q, q_uniform, rho32, rho64, what):
    """FP32 vertex charge against the FP64 oracle, per vertex.

    Every vertex: error <= 1e-6 times the total |charge| of the particles
    whose leaf has the vertex as a corner.  A particle's FP32 position carries
    an absolute rounding of its offset, so each of its weights carries an
    absolute error; a vertex reached only by the tip of a few weights holds a
    tiny charge whose plain relative error measures that tip's rounding.
    Populated vertices (touched by at least 64 particles; in the uniform
    plasmas every vertex): plain relative error |rho32 - rho64| / |rho64|
    <= 1e-6.  Returns the largest plain relative error over those."""
    w, vtx = o.weights(x)
    qa = np.abs(q) if q is not None else np.full(x.shape[1], abs(q_uniform))
    touch = np.bincount(vtx.ravel(), weights=np.repeat(qa, vtx.shape[1]), minlength=o.n_vertices)
    count = np.bincount(vtx.ravel(), minlength=o.n_vertices)
    err = np.abs(rho32 - rho64)
    pop = (count >= POPULATED) & (rho64 != 0)
    rel = err[pop] / np.abs(rho64[pop]) if pop.any() else np.zeros(1)
    assert rel.max() <= RHO_F32, (what, "populated vertex", float(rel.max()))
    assert (err <= RHO_F32 * touch).all(), (what, "vertex against its particles' charge",
                                             float((err / np.maximum(touch, 1e-300)).max()))
    return float(rel.max())
