"""Colour difference of two renders, FP64 reference (test infrastructure only).

The renders are compared by the CIE's year-2000 colour difference (CIEDE2000,
CIE publication 142-2001), the measure the paper's image-quality comparison
uses (a difference of 1 is just noticeable; the paper accepts up to 5).  Steps,
each in its published form:
  1. premultiplied RGBA composited over a background colour: c = C + (1 - A) bg;
  2. c read as sRGB-encoded (IEC 61966-2-1): linear = c/12.92 for c <= 0.04045,
     ((c + 0.055)/1.055)^2.4 above;
  3. linear sRGB to CIE XYZ with the sRGB primaries and the D65 white (the
     matrix of IEC 61966-2-1);
  4. XYZ to CIELAB relative to the D65 white (CIE 15: f(t) = t^(1/3) above
     (6/29)^3, t/(3 (6/29)^2) + 4/29 below);
  5. CIEDE2000 with k_L = k_C = k_H = 1.
Nothing here is shared with the GPU library.
"""
import numpy as np

# IEC 61966-2-1 (sRGB) linear RGB -> XYZ, D65
_M = np.array([[0.4124, 0.3576, 0.1805],
               [0.2126, 0.7152, 0.0722],
               [0.0193, 0.1192, 0.9505]])
_WHITE = _M @ np.ones(3)          # XYZ of RGB (1, 1, 1): the D65 white of the matrix


def composite(rgba, background=(1.0, 1.0, 1.0)):
    rgba = np.asarray(rgba, dtype=np.float64).reshape(-1, 4)
    bg = np.asarray(background, dtype=np.float64)
    return rgba[:, :3] + (1.0 - rgba[:, 3:4]) * bg[None, :]


def srgb_to_lab(rgb):
    c = np.clip(np.asarray(rgb, dtype=np.float64).reshape(-1, 3), 0.0, 1.0)
    lin = np.where(c <= 0.04045, c / 12.92, ((c + 0.055) / 1.055) ** 2.4)
    xyz = lin @ _M.T
    t = xyz / _WHITE[None, :]
    d = 6.0 / 29.0
    f = np.where(t > d ** 3, np.cbrt(t), t / (3 * d * d) + 4.0 / 29.0)
    L = 116.0 * f[:, 1] - 16.0
    a = 500.0 * (f[:, 0] - f[:, 1])
    b = 200.0 * (f[:, 1] - f[:, 2])
    return np.stack([L, a, b], 1)


def ciede2000(lab1, lab2):
    """CIEDE2000 between rows of CIELAB colours (k_L = k_C = k_H = 1)."""
    L1, a1, b1 = np.asarray(lab1, dtype=np.float64).reshape(-1, 3).T
    L2, a2, b2 = np.asarray(lab2, dtype=np.float64).reshape(-1, 3).T
    C1, C2 = np.hypot(a1, b1), np.hypot(a2, b2)
    Cm = 0.5 * (C1 + C2)
    G = 0.5 * (1.0 - np.sqrt(Cm ** 7 / (Cm ** 7 + 25.0 ** 7)))
    a1p, a2p = (1.0 + G) * a1, (1.0 + G) * a2
    C1p, C2p = np.hypot(a1p, b1), np.hypot(a2p, b2)
    h1p = np.where((a1p == 0) & (b1 == 0), 0.0, np.degrees(np.arctan2(b1, a1p)) % 360.0)
    h2p = np.where((a2p == 0) & (b2 == 0), 0.0, np.degrees(np.arctan2(b2, a2p)) % 360.0)
    dLp = L2 - L1
    dCp = C2p - C1p
    dh = h2p - h1p
    dh = np.where(dh > 180.0, dh - 360.0, np.where(dh < -180.0, dh + 360.0, dh))
    dh = np.where(C1p * C2p == 0, 0.0, dh)
    dHp = 2.0 * np.sqrt(C1p * C2p) * np.sin(np.radians(dh) / 2.0)
    Lpm = 0.5 * (L1 + L2)
    Cpm = 0.5 * (C1p + C2p)
    hsum = h1p + h2p
    hpm = np.where(C1p * C2p == 0, hsum,
                   np.where(np.abs(h1p - h2p) <= 180.0, 0.5 * hsum,
                            np.where(hsum < 360.0, 0.5 * (hsum + 360.0), 0.5 * (hsum - 360.0))))
    T = (1.0 - 0.17 * np.cos(np.radians(hpm - 30.0)) + 0.24 * np.cos(np.radians(2.0 * hpm)) +
         0.32 * np.cos(np.radians(3.0 * hpm + 6.0)) - 0.20 * np.cos(np.radians(4.0 * hpm - 63.0)))
    dtheta = 30.0 * np.exp(-(((hpm - 275.0) / 25.0) ** 2))
    RC = 2.0 * np.sqrt(Cpm ** 7 / (Cpm ** 7 + 25.0 ** 7))
    SL = 1.0 + 0.015 * (Lpm - 50.0) ** 2 / np.sqrt(20.0 + (Lpm - 50.0) ** 2)
    SC = 1.0 + 0.045 * Cpm
    SH = 1.0 + 0.015 * Cpm * T
    RT = -np.sin(np.radians(2.0 * dtheta)) * RC
    return np.sqrt((dLp / SL) ** 2 + (dCp / SC) ** 2 + (dHp / SH) ** 2 + RT * (dCp / SC) * (dHp / SH))


def delta_e_images(rgba_a, rgba_b, background=(1.0, 1.0, 1.0)):
    """Per pixel CIEDE2000 between two premultiplied RGBA images over `background`."""
    return ciede2000(srgb_to_lab(composite(rgba_a, background)), srgb_to_lab(composite(rgba_b, background)))
