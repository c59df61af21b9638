"""Points of a depth-map pair in FP64 (oracle; test infrastructure only).

Sec. III-C.1 builds a submap by unprojecting its frames' predicted depths with
the predicted cameras. For pair k, stored element i (pixel j = i - offsets[k]
of the pair) lies in shared frame f = j // frame_pixels at column
(j mod frame_pixels) mod width and row (j mod frame_pixels) // width, and

    p = R_p,f (d_p K^{-1} [col, row, 1]) + t_p,f,   q = R_q,f (d_q K^{-1} [col, row, 1]) + t_q,f

with K^{-1} [col, row, 1] = ((col - cx)/fx, (row - cy)/fy, 1) per camera. The
alignment oracle then runs on (p, q, c) unchanged.
"""

import numpy as np


def pair_geometry_valid(rec, n):
    W, HW, nf = int(rec["width"]), int(rec["frame_pixels"]), int(rec["n_frames"])
    return (W >= 1 and HW >= W and HW % W == 0 and 1 <= nf <= 4 and int(rec["reserved"]) == 0
            and n <= nf * HW)


def unproject_pair(dp, dq, rec):
    """(p, q) as (n, 3) float64 arrays for one pair's depth elements."""
    n = len(dp)
    W, HW = int(rec["width"]), int(rec["frame_pixels"])
    j = np.arange(n)
    f = j // HW
    pix = j - f * HW
    row, col = pix // W, pix - (pix // W) * W
    out = []
    for d, side in ((np.asarray(dp, np.float64), "p"), (np.asarray(dq, np.float64), "q")):
        x = np.zeros((n, 3))
        for fr in np.unique(f):
            cam = rec[side][fr]
            sel = f == fr
            ray = np.stack([(col[sel] - float(cam["cx"])) / float(cam["fx"]),
                            (row[sel] - float(cam["cy"])) / float(cam["fy"]), np.ones(int(sel.sum()))], 1)
            R = np.asarray(cam["R"], np.float64).reshape(3, 3)
            x[sel] = (d[sel, None] * ray) @ R.T + np.asarray(cam["t"], np.float64)
        out.append(x)
    return out[0], out[1]
