"""Converters from the seeded workload records to the oracle's types."""

import numpy as np

from oracle import bspline as ob
from oracle import raycast as orc


def oracle_model(spec, ctrl=None):
    """Oracle model of a spec; with ``ctrl`` given (de-quantised values) the
    caller sets the matching weights of a rational model."""
    w = getattr(spec, "weights", None)
    return ob.Model(tuple(spec.degree), tuple(np.asarray(k, dtype=np.float64) for k in spec.knots),
                    np.asarray(spec.ctrl if ctrl is None else ctrl, dtype=np.float64),
                    np.asarray(spec.lo, dtype=np.float64), np.asarray(spec.hi, dtype=np.float64),
                    weights=None if (ctrl is not None or w is None) else np.asarray(w, np.float64))


def oracle_camera(c):
    return orc.Camera(c.kind, tuple(c.eye), tuple(c.target), tuple(c.up), c.width, c.height,
                      c.fov_y_deg, c.ortho_half_w, c.ortho_half_h)


def oracle_tf(t):
    return orc.TransferFunction(np.asarray(t.table, dtype=np.float32), float(t.v_lo), float(t.v_hi))


def oracle_params(p):
    return orc.RenderParams(step=p.step, ert_alpha=p.ert_alpha, shading=p.shading, ka=p.ka,
                            kd=p.kd, ks=p.ks, shininess=p.shininess, headlight=p.headlight,
                            light_dir=tuple(p.light_dir))


def oracle_workload(w):
    return oracle_model(w.model), oracle_camera(w.camera), oracle_tf(w.tf), oracle_params(w.params)
