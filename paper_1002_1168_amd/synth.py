"""Seeded synthetic video-object sequences: composited 8-bit luma plus one
binary alpha plane per video object plane (VOP).

The paper evaluates on four natural QCIF test sequences (Section 4) that are
not available here; these generators stand in for them.  Every sequence is a
pure function of its seed, so the GPU path and the CPU oracle are fed the very
same bytes.  This module holds input generation only: it contains none of the
motion-estimation arithmetic.

Recipe (shared by every workload):
  * texture  = i.i.d. uniform bytes, separable Gaussian blur (sigma 2 px,
    radius 6, integer taps summing to 256), linear stretch to [16, 235];
  * shapes   = ellipse or convex polygon (5..7 vertices) tested at pixel
    centres (even-odd rule for polygons) -> binary alpha {0, 255};
  * compositing: background first, then VOP 0, 1, ... (a later VOP is in
    front); alpha of VOP k = its visible pixels only;
  * objects move rigidly; integer positions render texels exactly, real
    positions (sub-pixel motion) render by bilinear interpolation;
  * per-frame additive noise round(N(0, sigma)) clipped to [0, 255].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

QCIF = (176, 144)
CIF = (352, 288)
CIF4 = (704, 576)
HD1088 = (1920, 1088)


@dataclass
class Sequence:
    """One video stream: ``luma[F,H,W]`` u8 and ``alpha[V,F,H,W]`` u8 (0/255).

    ``V == 0`` means a rectangular (shape-less) sequence.
    """

    luma: np.ndarray
    alpha: np.ndarray
    search_range: int
    half_pel: bool = False
    name: str = ""
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def frames(self) -> int:
        return int(self.luma.shape[0])

    @property
    def height(self) -> int:
        return int(self.luma.shape[1])

    @property
    def width(self) -> int:
        return int(self.luma.shape[2])

    @property
    def vops(self) -> int:
        return int(self.alpha.shape[0])

    @property
    def mbs_per_frame(self) -> int:
        return (self.width // 16) * (self.height // 16)


# ----------------------------------------------------------------- texture
def gaussian_taps(sigma: float = 2.0, radius: int = 6, scale: int = 256) -> np.ndarray:
    k = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-k * k / (2.0 * sigma * sigma))
    w /= w.sum()
    t = np.rint(w * scale).astype(np.int64)
    t[radius] += scale - int(t.sum())
    return t


def smoothed_noise(rng: np.random.Generator, h: int, w: int,
                   sigma: float = 2.0, radius: int = 6) -> np.ndarray:
    """Blurred uniform noise stretched to [16, 235], shape (h, w), u8."""
    raw = rng.integers(0, 256, size=(h + 2 * radius, w + 2 * radius), dtype=np.int64)
    taps = gaussian_taps(sigma, radius)
    n = 2 * radius + 1
    tmp = np.zeros((h + 2 * radius, w), dtype=np.int64)
    for i in range(n):
        tmp += taps[i] * raw[:, i:i + w]
    tmp = (tmp + 128) >> 8
    out = np.zeros((h, w), dtype=np.int64)
    for i in range(n):
        out += taps[i] * tmp[i:i + h, :]
    out = (out + 128) >> 8
    lo, hi = int(out.min()), int(out.max())
    span = max(hi - lo, 1)
    return (16 + (2 * (out - lo) * 219 + span) // (2 * span)).astype(np.uint8)


# ------------------------------------------------------------------ shapes
@dataclass
class Shape:
    kind: str                      # "ellipse" | "polygon"
    a: float = 0.0                 # ellipse semi-axis along x
    b: float = 0.0                 # ellipse semi-axis along y
    verts: np.ndarray | None = None  # polygon vertices relative to the centre

    @property
    def radius(self) -> float:
        if self.kind == "ellipse":
            return float(max(self.a, self.b))
        return float(np.sqrt((self.verts ** 2).sum(axis=1)).max())

    def inside(self, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
        """Pixel-centre inside test; xs, ys are offsets from the centre."""
        if self.kind == "ellipse":
            return (xs / self.a) ** 2 + (ys / self.b) ** 2 <= 1.0
        v = self.verts
        k = v.shape[0]
        res = np.zeros(np.broadcast(xs, ys).shape, dtype=bool)
        for i in range(k):
            x1, y1 = v[i]
            x2, y2 = v[(i + 1) % k]
            if y1 == y2:
                continue
            cross = (y1 > ys) != (y2 > ys)
            xint = (x2 - x1) * (ys - y1) / (y2 - y1) + x1
            res ^= cross & (xs < xint)
        return res


def ellipse(a: float, b: float) -> Shape:
    return Shape("ellipse", a=float(a), b=float(b))


def random_polygon(rng: np.random.Generator, r: float) -> Shape:
    k = int(rng.integers(5, 8))
    ang = np.sort(rng.uniform(0.0, 2.0 * np.pi, size=k))
    # keep the polygon convex: vertices on a circle, radii jittered mildly
    rad = r * rng.uniform(0.85, 1.0, size=k)
    verts = np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)
    # convex hull to guarantee convexity after the radius jitter
    verts = _convex_hull(verts)
    return Shape("polygon", verts=verts)


def _convex_hull(p: np.ndarray) -> np.ndarray:
    pts = sorted(map(tuple, p))

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for q in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], q) <= 0:
            lower.pop()
        lower.append(q)
    for q in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], q) <= 0:
            upper.pop()
        upper.append(q)
    return np.array(lower[:-1] + upper[:-1], dtype=np.float64)


def random_shape(rng: np.random.Generator, r: float) -> Shape:
    if rng.random() < 0.5:
        return ellipse(r, r * rng.uniform(0.55, 1.0))
    return random_polygon(rng, r)


# ----------------------------------------------------------------- objects
@dataclass
class VideoObject:
    shape: Shape
    texture: np.ndarray            # square canvas, centred on the object
    pos: np.ndarray                # (F, 2) centre positions (x, y)


def _track(rng, frames, start, lo, hi, velocity_fn):
    """Positions over time with reflection at [lo, hi] per axis."""
    pos = np.zeros((frames, 2), dtype=np.float64)
    p = np.array(start, dtype=np.float64)
    v = None
    for t in range(frames):
        pos[t] = p
        v, step = velocity_fn(v)
        q = p + step
        for ax in range(2):
            if q[ax] < lo[ax]:
                q[ax] = 2 * lo[ax] - q[ax]
                v = None if v is None else _flip(v, ax)
            elif q[ax] > hi[ax]:
                q[ax] = 2 * hi[ax] - q[ax]
                v = None if v is None else _flip(v, ax)
            q[ax] = min(max(q[ax], lo[ax]), hi[ax])
        p = q
    return pos


def _flip(v, ax):
    v = np.array(v, dtype=np.float64)
    v[ax] = -v[ax]
    return v


def make_object(rng, shape: Shape, frames: int, W: int, H: int, motion: str,
                vmax: float) -> VideoObject:
    r = shape.radius
    half = int(np.ceil(r)) + 4
    tex = smoothed_noise(rng, 2 * half + 2, 2 * half + 2)
    lo = np.array([r + 1.0, r + 1.0])
    hi = np.array([W - r - 1.0, H - r - 1.0])
    hi = np.maximum(hi, lo)
    if motion == "subpel":
        start = rng.uniform(lo, hi)
    else:
        start = np.array([rng.integers(int(np.ceil(lo[0])), int(np.floor(hi[0])) + 1),
                          rng.integers(int(np.ceil(lo[1])), int(np.floor(hi[1])) + 1)],
                         dtype=np.float64)
    vm = int(vmax)
    if motion == "random_int":        # fresh integer step every frame
        def vel(v):
            s = rng.integers(-vm, vm + 1, size=2).astype(np.float64)
            return None, s
    elif motion == "const_jitter":    # constant velocity + per-frame jitter
        base = rng.integers(-vm, vm + 1, size=2).astype(np.float64)

        def vel(v):
            v = base if v is None else v
            j = rng.integers(-2, 3, size=2).astype(np.float64)
            return v, v + j
    elif motion == "const_int":
        base = rng.integers(-vm, vm + 1, size=2).astype(np.float64)

        def vel(v):
            v = base if v is None else v
            return v, v
    elif motion == "subpel":
        base = rng.uniform(-vmax, vmax, size=2)

        def vel(v):
            v = base if v is None else v
            return v, v
    else:
        raise ValueError(motion)
    pos = _track(rng, frames, start, lo, hi, vel)
    if motion != "subpel":
        pos = np.rint(pos)
    return VideoObject(shape, tex, pos)


def render(rng, W, H, frames, objects, bg, pan, noise_sigma) -> tuple[np.ndarray, np.ndarray]:
    """Composite ``objects`` over the background canvas ``bg``.

    ``pan`` is (F, 2) integer background offsets.  Returns (luma, alpha).
    """
    V = len(objects)
    luma = np.empty((frames, H, W), dtype=np.uint8)
    alpha = np.zeros((V, frames, H, W), dtype=np.uint8)
    for t in range(frames):
        ox, oy = int(pan[t, 0]), int(pan[t, 1])
        frame = bg[oy:oy + H, ox:ox + W].astype(np.float64)
        owner = np.full((H, W), -1, dtype=np.int16)
        for k, ob in enumerate(objects):
            cx, cy = ob.pos[t]
            half = ob.texture.shape[0] // 2 - 1
            r = ob.shape.radius
            x0 = max(int(np.floor(cx - r)) - 1, 0)
            x1 = min(int(np.ceil(cx + r)) + 2, W)
            y0 = max(int(np.floor(cy - r)) - 1, 0)
            y1 = min(int(np.ceil(cy + r)) + 2, H)
            if x1 <= x0 or y1 <= y0:
                continue
            xs = np.arange(x0, x1, dtype=np.float64) + 0.5 - cx
            ys = np.arange(y0, y1, dtype=np.float64) + 0.5 - cy
            XS, YS = np.meshgrid(xs, ys)
            m = ob.shape.inside(XS, YS)
            # texel i sits at pixel x = cx + i - half: an integer centre
            # copies texels exactly, a real centre interpolates bilinearly
            u = XS - 0.5 + half
            w = YS - 0.5 + half
            iu = np.floor(u).astype(np.int64)
            iw = np.floor(w).astype(np.int64)
            fu = u - iu
            fw = w - iw
            tx = ob.texture.astype(np.float64)
            iu = np.clip(iu, 0, tx.shape[1] - 2)
            iw = np.clip(iw, 0, tx.shape[0] - 2)
            val = ((1 - fu) * (1 - fw) * tx[iw, iu] + fu * (1 - fw) * tx[iw, iu + 1]
                   + (1 - fu) * fw * tx[iw + 1, iu] + fu * fw * tx[iw + 1, iu + 1])
            sub = frame[y0:y1, x0:x1]
            sub[m] = np.rint(val[m])
            osub = owner[y0:y1, x0:x1]
            osub[m] = k
        for k in range(V):
            alpha[k, t] = np.where(owner == k, 255, 0).astype(np.uint8)
        if noise_sigma > 0:
            frame = frame + np.rint(rng.normal(0.0, noise_sigma, size=(H, W)))
        luma[t] = np.clip(frame, 0, 255).astype(np.uint8)
    return luma, alpha


def _background(rng, W, H, frames, pan_speed):
    extra = abs(pan_speed) * frames + 2
    bg = smoothed_noise(rng, H + 2, W + extra)
    pan = np.zeros((frames, 2), dtype=np.int64)
    for t in range(frames):
        pan[t, 0] = (t * pan_speed) if pan_speed >= 0 else (extra - 2 + t * pan_speed)
    return bg, pan


def make_sequence(seed, W, H, frames, shapes_fn, motion, vmax, search_range,
                  pan_speed=0, noise_sigma=2.0, half_pel=False, name="") -> Sequence:
    rng = np.random.default_rng(seed)
    bg, pan = _background(rng, W, H, frames, pan_speed)
    shapes = shapes_fn(rng)
    objs = [make_object(rng, s, frames, W, H, motion, vmax) for s in shapes]
    luma, alpha = render(rng, W, H, frames, objs, bg, pan, noise_sigma)
    return Sequence(luma, alpha, search_range, half_pel, name, int(seed),
                    meta={"motion": motion, "vmax": vmax, "pan": pan_speed,
                          "noise_sigma": noise_sigma,
                          "positions": [o.pos.tolist() for o in objs]})


# ------------------------------------------------------------- workloads
def qcif_ellipse(seed: int = 1, frames: int = 10) -> Sequence:
    """QCIF 176x144, one ellipse VOP (semi-axes 40x28), integer step
    U{-4..4}^2 per frame reflected at the borders, static background,
    N(0, 2) noise, search range 7."""
    W, H = QCIF
    return make_sequence(seed, W, H, frames, lambda rng: [ellipse(40, 28)],
                         "random_int", 4, 7, pan_speed=0, name="qcif_ellipse")


def cif_two_vops(seed: int = 2, frames: int = 300) -> Sequence:
    """CIF 352x288, a polygon and an ellipse VOP with constant integer
    velocity U{-3..3}^2 plus jitter U{-2..2}^2 per frame, mutual occlusion,
    background panning 1 px/frame, N(0, 2) noise, search range 16."""
    W, H = CIF

    def shapes(rng):
        return [random_polygon(rng, 64.0), ellipse(70, 50)]

    return make_sequence(seed, W, H, frames, shapes, "const_jitter", 3, 16,
                         pan_speed=1, name="cif_two_vops")


def _random_vop_shapes(lo_n, hi_n, W, H, rmin, rmax):
    def shapes(rng):
        n = int(rng.integers(lo_n, hi_n + 1))
        m = min(W, H)
        return [random_shape(rng, rng.uniform(rmin, rmax) * m) for _ in range(n)]
    return shapes


def mixed_streams(seed: int = 3, frames: int = 30, counts=(24, 24, 16)) -> list[Sequence]:
    """64 streams (24 QCIF, 24 CIF, 16 4CIF), 1..4 VOPs each, integer
    velocities U{-8..8}^2, search range 16."""
    out = []
    sizes = [QCIF] * counts[0] + [CIF] * counts[1] + [CIF4] * counts[2]
    ss = np.random.SeedSequence(seed)
    for i, (W, H) in enumerate(sizes):
        s = int(ss.spawn(1)[0].generate_state(1)[0])
        out.append(make_sequence(s, W, H, frames,
                                 _random_vop_shapes(1, 4, W, H, 0.12, 0.3),
                                 "const_int", 8, 16, pan_speed=0,
                                 name=f"mixed{i}_{W}x{H}"))
    return out


def cif_training_set(seed: int, count: int, frames: int = 30) -> list[Sequence]:
    """CIF sequences in the two-VOP style but with 1..4 random VOPs."""
    W, H = CIF
    ss = np.random.SeedSequence(seed)
    out = []
    for i in range(count):
        s = int(ss.spawn(1)[0].generate_state(1)[0])
        out.append(make_sequence(s, W, H, frames,
                                 _random_vop_shapes(1, 4, W, H, 0.15, 0.25),
                                 "const_jitter", 3, 16, pan_speed=1,
                                 name=f"cif_train{i}"))
    return out


def _hd_one(args) -> Sequence:
    s, frames, i = args
    W, H = HD1088
    return make_sequence(s, W, H, frames, _random_vop_shapes(3, 6, W, H, 0.08, 0.25),
                         "subpel", 24.0, 32, pan_speed=0, half_pel=True, name=f"hd{i}")


def hd_streams(seed: int = 5, frames: int = 60, streams: int = 8, workers: int = 1) -> list[Sequence]:
    """1920x1088 streams, 3..6 VOPs with occlusion, real velocities
    U[-24, 24]^2 rendered bilinearly, search range 32, half-pel.  Each
    stream is a pure function of its own seed, so ``workers`` > 1 renders
    the streams in forked processes with the same bytes."""
    ss = np.random.SeedSequence(seed)
    args = [(int(ss.spawn(1)[0].generate_state(1)[0]), frames, i) for i in range(streams)]
    if workers <= 1 or streams <= 1:
        return [_hd_one(a) for a in args]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(workers, streams)) as pool:
        return pool.map(_hd_one, args, chunksize=1)


def random_frames(seed: int, W: int, H: int, frames: int = 2, vops: int = 0,
                  search_range: int = 4) -> Sequence:
    """Unstructured uniform noise frames (and random blob alphas) for
    brute-force checks on tiny inputs."""
    rng = np.random.default_rng(seed)
    luma = rng.integers(0, 256, size=(frames, H, W), dtype=np.uint8)
    alpha = np.zeros((vops, frames, H, W), dtype=np.uint8)
    for k in range(vops):
        for t in range(frames):
            cx, cy = rng.uniform(0, W), rng.uniform(0, H)
            a, b = rng.uniform(6, W / 2), rng.uniform(6, H / 2)
            ys, xs = np.mgrid[0:H, 0:W]
            m = ((xs + 0.5 - cx) / a) ** 2 + ((ys + 0.5 - cy) / b) ** 2 <= 1.0
            alpha[k, t] = np.where(m, 255, 0)
    return Sequence(luma, alpha, search_range, False, "random", int(seed))


# ---------------------------------------------------------------- network
# Fan-ins of the proposal network's three 3x3 convolutions (2, 32, 32 input
# channels) and their output channels, in parameter-vector order:
# W1 (32,3,3,2) | b1 (32) | W2 (32,3,3,32) | b2 (32) | W3 (2,3,3,32) | b3 (2).
_NET_TENSORS = ((32 * 9 * 2, 9 * 2, 2.0), (32, 0, 0.0), (32 * 9 * 32, 9 * 32, 2.0), (32, 0, 0.0),
                (2 * 9 * 32, 9 * 32, 0.5), (2, 0, 0.0))


def net_init(seed: int) -> np.ndarray:
    """Seeded initial weights of the proposal network (float32): normal
    weights with variance gain / fan-in, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for n, fan_in, gain in _NET_TENSORS:
        if fan_in:
            parts.append(rng.normal(0.0, np.sqrt(gain / fan_in), size=n))
        else:
            parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)
