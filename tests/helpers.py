"""Small numpy helpers shared by the tests (no renderer arithmetic)."""
import numpy as np


def to_clip(pos, mvp):
    """[V,3] world positions, [B,4,4] matrices -> [B,V,4] clip coordinates (float32)."""
    p = np.concatenate([np.asarray(pos, np.float64), np.ones((len(pos), 1))], 1)
    m = np.asarray(mvp, np.float64)
    if m.ndim == 2:
        m = m[None]
    return np.einsum("bij,vj->bvi", m, p).astype(np.float32)


def screen_to_clip(xy_px, H, W, z=0.5, w=1.0):
    """Pixel-space (x right, y down) positions -> clip coordinates with given z/w and w."""
    xy = np.asarray(xy_px, np.float64)
    xn = xy[:, 0] / (W / 2.0) - 1.0
    yn = 1.0 - xy[:, 1] / (H / 2.0)
    z = np.broadcast_to(np.asarray(z, np.float64), (len(xy),))
    w = np.broadcast_to(np.asarray(w, np.float64), (len(xy),))
    return np.stack([xn * w, yn * w, z * w, w], 1).astype(np.float32)


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    n = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (n if n > 0 else 1.0)
