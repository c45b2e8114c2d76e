"""Camera quantisation for the oracle, in exact arithmetic (TEST
INFRASTRUCTURE ONLY; see the package docstring).

A camera description (eye, target, up, vertical field of view or
orthographic height, W x H pixels) becomes the integer ray record that both
renderers consume: positions and direction steps in units of 2^-28 of the
box.  The paper fixes only that one ray is shot per pixel (Sec. 2.2) and
that the camera's pixel size decides the deepest level read (Sec. 2); the
record below is the reading taken for the rest.

Definition (real numbers, no rounding until the end):
  f  = target - eye                      (view vector)
  g  = up x f                            (image-plane x axis, unnormalised)
  h  = f x g                             (image-plane y axis, unnormalised;
                                          |h| = |f| |g| because g is normal to f)
  s  = tan(fov_y / 2) / H                (perspective: half-pixel step at unit
                                          distance along the unit view vector)
     = ortho_height / (2 H)              (orthographic: half-pixel step in box units)
  O  = rne(2^28 eye)
  F  = rne(2^28 f / |f|)
  U  = rne(2^28 s g / |g|)
  V  = rne(2^28 s h / (|f| |g|))
with rne = round to the nearest integer, ties to even.  Pixel (i, j) then
has the ray O + t (F + aU + bV) (perspective) or (O + aU + bV) + t F
(orthographic) with a = 2i + 1 - W, b = 2j + 1 - H: through the pixel
centre, j = 0 at the bottom of the image.

Automatic maximum level: the pixel footprint is p = 2 |f| tan(fov_y/2) / H
(perspective, at the target distance) or ortho_height / H; the level is the
smallest L >= 0 with 2^-L <= p, plus level_bias, clamped to [0, 24] and to
the tree's deepest level.

The inputs are doubles, hence exact rationals.  Every record component is
x = q / sqrt(r) or x = q * tan(theta) / sqrt(r) with rationals q, r: the
square roots are evaluated in 90-digit decimal arithmetic and the rounding
(and, where x is algebraic, a tie) is then decided exactly by comparing
squares of rationals.  With a tangent the value is transcendental for every
theta != 0, so no tie can occur, and the 90 digits decide the rounding.
This formulation (exact cross products, one square root per component)
shares nothing with the library's floating-point evaluation of the same
definition.
"""
from __future__ import annotations

import math
from decimal import Decimal, localcontext
from fractions import Fraction
from typing import Optional, Sequence

FIX = 28
MAX_LEVEL = 24
_DIGITS = 90


class CameraError(ValueError):
    """The description cannot be quantised into a valid record."""


def _cross(a: Sequence[Fraction], b: Sequence[Fraction]):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _dot(a, b) -> Fraction:
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _dec(q: Fraction) -> Decimal:
    return Decimal(q.numerator) / Decimal(q.denominator)


def _rne_rational(x: Fraction) -> int:
    # Python's round() of a Fraction rounds half to even, exactly
    return int(round(x))


def _cmp_q_over_sqrt(q: Fraction, r: Fraction, m: Fraction) -> int:
    """Sign of q / sqrt(r) - m, exactly (r > 0)."""
    if q == 0 and m == 0:
        return 0
    if q >= 0 and m <= 0:
        return 1
    if q <= 0 and m >= 0:
        return -1
    # same sign: compare |q| / sqrt(r) with |m| through q^2 and m^2 r
    a, b = q * q, m * m * r
    c = (a > b) - (a < b)
    return c if q > 0 else -c


def _rne_q_over_sqrt(q: Fraction, r: Fraction) -> int:
    """rne(q / sqrt(r)) exactly, for rationals q and r > 0."""
    with localcontext() as ctx:
        ctx.prec = _DIGITS
        est = _dec(q) / _dec(r).sqrt()
    n = int(est.to_integral_value(rounding="ROUND_FLOOR"))
    # settle the floor exactly (the estimate is within 1e-80 of the value)
    while _cmp_q_over_sqrt(q, r, Fraction(n)) < 0:
        n -= 1
    while _cmp_q_over_sqrt(q, r, Fraction(n + 1)) >= 0:
        n += 1
    c = _cmp_q_over_sqrt(q, r, Fraction(2 * n + 1, 2))
    if c > 0 or (c == 0 and n % 2 == 1):
        return n + 1
    return n


def _tan(theta: Fraction) -> Decimal:
    """tan(theta) for 0 < theta < 1.5, by the Taylor series of sin and cos in
    high-precision decimal arithmetic."""
    with localcontext() as ctx:
        ctx.prec = _DIGITS + 20
        x = _dec(theta)
        x2 = x * x
        s, c = Decimal(0), Decimal(0)
        ts, tc = x, Decimal(1)
        k = 0
        eps = Decimal(10) ** (-(_DIGITS + 15))
        while abs(ts) > eps or abs(tc) > eps:
            s += ts
            c += tc
            ts = -ts * x2 / ((2 * k + 2) * (2 * k + 3))
            tc = -tc * x2 / ((2 * k + 1) * (2 * k + 2))
            k += 1
        return s / c


def _rne_tan_q_over_sqrt(t: Decimal, q: Fraction, r: Fraction) -> int:
    """rne(t q / sqrt(r)) with t = tan(theta) (transcendental: no tie)."""
    with localcontext() as ctx:
        ctx.prec = _DIGITS
        x = t * _dec(q) / _dec(r).sqrt()
        return int(x.to_integral_value(rounding="ROUND_HALF_EVEN"))


class Record:
    """The integer camera record (mirrors the C struct layout by field name)."""

    __slots__ = ("kind", "W", "H", "max_level", "O", "F", "U", "V")

    def __init__(self, kind, W, H, max_level, O, F, U, V):
        self.kind, self.W, self.H, self.max_level = int(kind), int(W), int(H), int(max_level)
        self.O, self.F, self.U, self.V = (list(map(int, O)), list(map(int, F)), list(map(int, U)),
                                          list(map(int, V)))

    def as_dict(self) -> dict:
        return dict(kind=self.kind, W=self.W, H=self.H, max_level=self.max_level, O=list(self.O),
                    F=list(self.F), U=list(self.U), V=list(self.V))


def _auto_level(foot_cmp) -> int:
    """Smallest L >= 0 with 2^-L <= p, given foot_cmp(L) = sign(2^-L - p)."""
    L = 0
    while L < 200 and foot_cmp(L) > 0:
        L += 1
    return L


def quantise(desc: dict, tree_lmax: Optional[int] = None) -> Record:
    """Record of a camera description (amrgen.camera dict).  Raises
    CameraError for descriptions the renderers reject: kind, W or H outside
    1..32768, non-finite vectors, eye == target, up parallel to the view,
    fov_y outside (0, 3), ortho_height <= 0, an explicit max_level above 24,
    or a record outside the integer ranges (origins in [-2^30, 2^30); every
    pixel's direction, or orthographic origin, inside those bounds)."""
    kind = desc["kind"]
    kind = {"persp": 0, "ortho": 1}.get(kind, kind)
    kind = int(kind)
    W, H = int(desc["W"]), int(desc["H"])
    if kind not in (0, 1):
        raise CameraError("kind")
    if not (1 <= W <= 32768 and 1 <= H <= 32768):
        raise CameraError("image size")
    vecs = [desc["eye"], desc["target"], desc["up"]]
    if not all(math.isfinite(float(v)) for vec in vecs for v in vec):
        raise CameraError("non-finite vector")
    eye = [Fraction(float(v)) for v in desc["eye"]]
    tgt = [Fraction(float(v)) for v in desc["target"]]
    up = [Fraction(float(v)) for v in desc["up"]]
    f = [tgt[k] - eye[k] for k in range(3)]
    ff = _dot(f, f)
    if ff == 0:
        raise CameraError("eye == target")
    g = _cross(up, f)
    gg = _dot(g, g)
    if gg == 0:
        raise CameraError("up parallel to the view")
    h = _cross(f, g)
    one = Fraction(1 << FIX)

    O = [_rne_rational(one * e) for e in eye]
    F = [_rne_q_over_sqrt(one * fk, ff) for fk in f]
    if kind == 0:
        fov = float(desc.get("fov_y", 0.0))
        if not (0.0 < fov < 3.0):
            raise CameraError("fov_y")
        theta = Fraction(fov) / 2
        t = _tan(theta)
        # U_k = 2^28 tan(theta) g_k / (H |g|);  V_k = 2^28 tan(theta) h_k / (H |f| |g|)
        U = [_rne_tan_q_over_sqrt(t, one * gk / H, gg) for gk in g]
        V = [_rne_tan_q_over_sqrt(t, one * hk / H, ff * gg) for hk in h]

        def foot_cmp(L):  # sign(2^-L - 2 |f| tan(theta) / H)
            with localcontext() as ctx:
                ctx.prec = _DIGITS
                p = 2 * _dec(ff).sqrt() * t / H
                lhs = Decimal(2) ** (-L)
                return (lhs > p) - (lhs < p)
    else:
        oh = float(desc.get("ortho_height", 0.0))
        if not (oh > 0.0 and math.isfinite(oh)):
            raise CameraError("ortho_height")
        s = Fraction(oh) / (2 * H)
        U = [_rne_q_over_sqrt(one * s * gk, gg) for gk in g]
        V = [_rne_q_over_sqrt(one * s * hk, ff * gg) for hk in h]
        p_ortho = Fraction(oh) / H

        def foot_cmp(L):
            lhs = Fraction(1, 1 << L)
            return (lhs > p_ortho) - (lhs < p_ortho)

    lim = 1 << 30
    for k in range(3):
        span = (W - 1) * abs(U[k]) + (H - 1) * abs(V[k])
        if not (-lim <= O[k] < lim):
            raise CameraError("eye outside [-4, 4) boxes")
        if kind == 0:
            if abs(F[k]) + span >= lim:
                raise CameraError("field of view too wide for the ray range")
        else:
            if not (-lim <= O[k] - span and O[k] + span < lim):
                raise CameraError("image plane outside [-4, 4) boxes")
            if abs(F[k]) >= lim:
                raise CameraError("direction out of range")

    ml = int(desc.get("max_level", -1))
    if ml >= 0:
        if ml > MAX_LEVEL:
            raise CameraError("max_level > 24")
        L = ml
    else:
        L = _auto_level(foot_cmp) + int(desc.get("level_bias", 0))
        L = max(0, min(L, MAX_LEVEL))
        if tree_lmax is not None and tree_lmax >= 0:
            L = min(L, int(tree_lmax))
    return Record(kind, W, H, L, O, F, U, V)
