"""Synthetic bundle-adjustment problems (camera simulation only).

Conventions shared by every workload:

* World frame has +z up. A keyframe pose is the 6-vector (omega, t) of a
  world-to-camera transform: a world point l maps to R(omega) l + t in the
  camera frame, with R(omega) the rotation whose axis-angle vector is omega.
* Camera axes: +x right, +y down, +z along the optical axis; pinhole
  intrinsics fx, fy, cx, cy; image width x height pixels.
* A point is visible from a keyframe when its camera depth exceeds 0.1 m
  and its noise-free projection falls inside the image.
* Measurements are noise-free projections plus N(0, sigma^2) pixel noise;
  an outlier measurement is replaced by a pixel drawn uniformly over the
  image (the inlier mask records which is which).
* Keyframe 0 starts at its true pose and carries a strong anchor prior
  (information 1e8); every other pose is perturbed by an axis-angle
  rotation error and a camera-centre error, landmarks by a position error.

Workload shapes follow the bundle-adjustment experiments of the paper
(Section 9: keyframes, landmarks and measurements of TUM-like sequences,
Table 1; outlier fractions of Section 9.4) with synthetic geometry standing in
for the TUM and KITTI data.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np
from scipy.spatial.transform import Rotation

DOWN = np.array([0.0, 0.0, -1.0])


@dataclass
class Camera:
    fx: float = 500.0
    fy: float = 500.0
    cx: float = 320.0
    cy: float = 240.0
    width: int = 640
    height: int = 480
    sigma: float = 1.0


@dataclass
class BAProblem:
    name: str
    cam: Camera
    kf_true: np.ndarray          # [Nk, 6] (omega, t), world -> camera
    lm_true: np.ndarray          # [Nl, 3]
    kf_init: np.ndarray          # [Nk, 6]
    lm_init: np.ndarray          # [Nl, 3]
    factor_kf: np.ndarray        # [Nf] int32
    factor_lm: np.ndarray        # [Nf] int32
    z: np.ndarray                # [Nf, 2] measured pixels
    z_true: np.ndarray           # [Nf, 2] noise-free projections of the truth
    inlier: np.ndarray           # [Nf] bool
    kf_anchor_info: np.ndarray   # [Nk] >0: strong isotropic prior at the init
    meta: dict = field(default_factory=dict)

    @property
    def n_keyframes(self) -> int:
        return int(self.kf_true.shape[0])

    @property
    def n_landmarks(self) -> int:
        return int(self.lm_true.shape[0])

    @property
    def n_factors(self) -> int:
        return int(self.factor_kf.shape[0])

    def cam_array(self) -> np.ndarray:
        c = self.cam
        return np.array([c.fx, c.fy, c.cx, c.cy, c.sigma], dtype=np.float64)


# ----------------------------------------------------------------------------
# camera simulation helpers
# ----------------------------------------------------------------------------

def _rotmat(omega: np.ndarray) -> np.ndarray:
    return Rotation.from_rotvec(np.atleast_2d(omega)).as_matrix()


def _pose_looking(centre: np.ndarray, fwd: np.ndarray) -> np.ndarray:
    """World->camera pose of a camera at `centre` whose optical axis is `fwd`
    and whose image y axis points as close to world-down as possible."""
    zc = fwd / np.linalg.norm(fwd)
    yc = DOWN - zc * (DOWN @ zc)
    yc /= np.linalg.norm(yc)
    xc = np.cross(yc, zc)
    r_cw = np.stack([xc, yc, zc], axis=1)        # camera -> world (columns)
    r_wc = r_cw.T                                # world -> camera
    omega = Rotation.from_matrix(r_wc).as_rotvec()
    t = -r_wc @ centre
    return np.concatenate([omega, t])


def _camera_points(kf: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Points [N,3] in the frames of keyframes kf [K,6] -> [N, K, 3]."""
    rot = _rotmat(kf[:, :3])                     # [K,3,3]
    return np.einsum("kij,nj->nki", rot, pts) + kf[None, :, 3:]


def _pixels(cam: Camera, pc: np.ndarray) -> np.ndarray:
    u = cam.fx * pc[..., 0] / pc[..., 2] + cam.cx
    v = cam.fy * pc[..., 1] / pc[..., 2] + cam.cy
    return np.stack([u, v], axis=-1)


def _visible(cam: Camera, pc: np.ndarray) -> np.ndarray:
    depth_ok = pc[..., 2] > 0.1
    with np.errstate(divide="ignore", invalid="ignore"):
        px = _pixels(cam, pc)
    inside = ((px[..., 0] >= 0) & (px[..., 0] < cam.width)
              & (px[..., 1] >= 0) & (px[..., 1] < cam.height))
    return depth_ok & inside


def _perturb(kf_true, lm_true, rng, rot_sigma, centre_sigma, lm_sigma):
    """Initial estimate: R_init = Exp(d_omega) R_true, centre + noise,
    landmarks + noise; keyframe 0 is left at its true pose."""
    nk = kf_true.shape[0]
    kf_init = kf_true.copy()
    for k in range(1, nk):
        r_true = _rotmat(kf_true[k, :3])[0]
        centre = -r_true.T @ kf_true[k, 3:]
        d_omega = rng.normal(0.0, rot_sigma, 3)
        r_init = _rotmat(d_omega)[0] @ r_true
        c_init = centre + rng.normal(0.0, centre_sigma, 3)
        kf_init[k, :3] = Rotation.from_matrix(r_init).as_rotvec()
        kf_init[k, 3:] = -r_init @ c_init
    lm_init = lm_true + rng.normal(0.0, lm_sigma, lm_true.shape)
    return kf_init, lm_init


def _measure(cam, kf_true, lm_true, fkf, flm, rng, outlier_frac):
    pc = (np.einsum("nij,nj->ni", _rotmat(kf_true[fkf, :3]), lm_true[flm])
          + kf_true[fkf, 3:])
    z_true = _pixels(cam, pc)
    z = z_true + rng.normal(0.0, cam.sigma, z_true.shape)
    inlier = np.ones(len(fkf), dtype=bool)
    n_out = int(round(outlier_frac * len(fkf)))
    if n_out > 0:
        idx = rng.choice(len(fkf), n_out, replace=False)
        inlier[idx] = False
        z[idx, 0] = rng.uniform(0, cam.width, n_out)
        z[idx, 1] = rng.uniform(0, cam.height, n_out)
    return z, z_true, inlier


def _assemble(name, cam, kf_true, lm_true, obs, rng, outlier_frac,
              rot_sigma, centre_sigma, lm_sigma, anchor=1e8, meta=None):
    fkf = np.concatenate([np.asarray(o, dtype=np.int32) for o in obs])
    flm = np.concatenate([np.full(len(o), j, dtype=np.int32)
                          for j, o in enumerate(obs)])
    z, z_true, inlier = _measure(cam, kf_true, lm_true, fkf, flm, rng,
                                 outlier_frac)
    kf_init, lm_init = _perturb(kf_true, lm_true, rng, rot_sigma,
                                centre_sigma, lm_sigma)
    anchor_info = np.zeros(kf_true.shape[0])
    anchor_info[0] = anchor
    return BAProblem(name, cam, kf_true, lm_true, kf_init, lm_init, fkf, flm,
                     z, z_true, inlier, anchor_info, dict(meta or {}))


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def make_config0(seed: int = 0, n_kf: int = 5, n_lm: int = 50,
                 radius: float = 2.0, sigma: float = 1.0,
                 camera: Camera | None = None) -> BAProblem:
    """Tiny loopy problem: keyframes evenly spaced on a horizontal circle,
    each facing the origin; landmarks uniform in a 1 m cube; each landmark
    observed by 3-5 distinct keyframes chosen among those that see it.
    `camera` replaces the default intrinsics (and its sigma the noise)."""
    rng = np.random.default_rng(seed)
    cam = camera if camera is not None else Camera(sigma=sigma)
    kf = []
    for i in range(n_kf):
        a = 2.0 * np.pi * i / n_kf
        c = radius * np.array([np.cos(a), np.sin(a), 0.0])
        kf.append(_pose_looking(c, -c))
    kf_true = np.array(kf)
    lm_true = np.zeros((n_lm, 3))
    obs = []
    for j in range(n_lm):
        while True:
            p = rng.uniform(-0.5, 0.5, 3)
            vis = np.flatnonzero(_visible(cam, _camera_points(kf_true, p[None]))[0])
            n = int(rng.integers(3, 6))
            if len(vis) >= n:
                break
        lm_true[j] = p
        obs.append(np.sort(rng.choice(vis, n, replace=False)))
    return _assemble("config0", cam, kf_true, lm_true, obs, rng, 0.0,
                     0.05, 0.05, 0.1)


def _walk(n_kf, rng, step=0.2, yaw_deg=5.0):
    centres = np.zeros((n_kf, 3))
    heading = np.zeros(n_kf)
    for i in range(1, n_kf):
        heading[i] = heading[i - 1] + np.deg2rad(rng.uniform(-yaw_deg, yaw_deg))
        centres[i] = centres[i - 1] + step * np.array(
            [np.cos(heading[i - 1]), np.sin(heading[i - 1]), 0.0])
    return centres, heading


def _count_sampler(kind, rng):
    if kind == "poisson":          # clamp(4 + Poisson(4), 4, 20)
        return lambda: int(np.clip(4 + rng.poisson(4.0), 4, 20))
    if kind == "powerlaw":         # P(n) ~ n^-2 on [2, 200]
        ns = np.arange(2, 201)
        p = ns.astype(np.float64) ** -2.0
        p /= p.sum()
        return lambda: int(rng.choice(ns, p=p))
    if kind == "uniform4_12":
        return lambda: int(rng.integers(4, 13))
    if kind == "sparse":           # clamp(2 + Poisson(2.6), 2, 20): ~4.6 per point
        return lambda: int(np.clip(2 + rng.poisson(2.6), 2, 20))
    raise ValueError(kind)


def make_random_walk(name: str, seed: int, n_kf: int, n_lm: int,
                     count: str = "poisson", outlier_frac: float = 0.0,
                     sigma: float = 1.0, depth=(2.0, 10.0),
                     max_tries: int = 30, min_obs: int = 2,
                     look_yaw_deg: float = 0.0,
                     rot_sigma: float = 0.0, centre_sigma: float = 0.07,
                     lm_sigma: float = 0.1, camera: Camera | None = None) -> BAProblem:
    """Random-walk trajectory (0.2 m steps, heading changes U(+-5 deg) per
    step), camera looking along the heading (rotated by look_yaw_deg). Each
    landmark is spawned from a random keyframe at a random pixel and depth
    U(depth), then observed by a sampled number of keyframes drawn among
    those that see it; when fewer keyframes see it than sampled, the
    landmark is re-spawned up to max_tries times and the count is then capped
    at the visible number.

    Initial estimate (Section 9.1 protocol): keyframe camera centres perturbed
    by N(0, 7 cm) per axis, orientations left at the truth, landmarks
    perturbed by N(0, 0.1 m) per axis; keyframe 0 exact and anchored.
    `camera` replaces the default intrinsics (and its sigma the noise)."""
    rng = np.random.default_rng(seed)
    cam = camera if camera is not None else Camera(sigma=sigma)
    centres, heading = _walk(n_kf, rng)
    yaw = heading + np.deg2rad(look_yaw_deg)
    kf_true = np.array([_pose_looking(c, np.array([np.cos(h), np.sin(h), 0.0]))
                        for c, h in zip(centres, yaw)])
    rots = _rotmat(kf_true[:, :3])
    sample_n = _count_sampler(count, rng)
    lm_true = np.zeros((n_lm, 3))
    obs = []
    n_capped = 0
    batch = 2048
    j = 0
    while j < n_lm:
        b = min(batch, n_lm - j) * 2
        src = rng.integers(0, n_kf, b)
        u = rng.uniform(0, cam.width, b)
        v = rng.uniform(0, cam.height, b)
        d = rng.uniform(depth[0], depth[1], b)
        pc = np.stack([(u - cam.cx) / cam.fx * d, (v - cam.cy) / cam.fy * d, d], 1)
        pw = np.einsum("nji,nj->ni", rots[src], pc - kf_true[src, 3:])
        vis = _visible(cam, _camera_points(kf_true, pw))
        cand = 0
        while j < n_lm and cand < b:
            n = sample_n()
            tries = 0
            while True:
                vk = np.flatnonzero(vis[cand])
                ok = len(vk) >= n
                if ok or tries >= max_tries or cand + 1 >= b:
                    break
                cand += 1
                tries += 1
            if len(vk) < max(min_obs, 1):
                cand += 1
                continue
            if len(vk) < n:
                n = len(vk)
                n_capped += 1
            lm_true[j] = pw[cand]
            obs.append(np.sort(rng.choice(vk, n, replace=False)))
            cand += 1
            j += 1
    meta = dict(n_capped=n_capped, count=count, outlier_frac=outlier_frac)
    return _assemble(name, cam, kf_true, lm_true, obs, rng, outlier_frac,
                     rot_sigma, centre_sigma, lm_sigma, meta=meta)


def make_config1(seed: int = 1) -> BAProblem:
    """Paper-scale problem: 125 keyframes, 1919 landmarks (the fr3teddy
    sizes of Table 1), 4-20 observations (8 on average), 3% outliers."""
    return make_random_walk("config1", seed, 125, 1919, "poisson", 0.03)


def make_config2(seed: int = 2) -> BAProblem:
    """Large problem: 1000 keyframes, 40000 landmarks, power-law
    observation counts (alpha 2, capped at 200), 5% outliers."""
    return make_random_walk("config2", seed, 1000, 40000, "powerlaw", 0.05,
                            min_obs=2)


def make_config3_problem(p: int, base_seed: int = 1000) -> BAProblem:
    """Problem p of the uneven batch: keyframes U{10..125}, landmarks
    U{100..2000}, 4-12 observations each, no outliers."""
    rng = np.random.default_rng(base_seed + p)
    nk = int(rng.integers(10, 126))
    nl = int(rng.integers(100, 2001))
    return make_random_walk(f"config3_p{p}", base_seed + p + 7_000_000, nk, nl,
                            "uniform4_12", 0.0)


def make_config3(n_problems: int = 256, base_seed: int = 1000):
    return [make_config3_problem(p, base_seed) for p in range(n_problems)]


def make_tree_chain(n_kf: int = 3, leaves_per_kf: int = 0, seed: int = 5,
                    sigma: float = 1.0) -> BAProblem:
    """Tree-shaped graph: keyframes kf0-l0-kf1-l1-...-kf(n-1) joined by one
    shared landmark each, plus `leaves_per_kf` landmarks seen by a single
    keyframe. The graph has no loops."""
    rng = np.random.default_rng(seed)
    cam = Camera(sigma=sigma)
    centres = np.array([[0.3 * i, 0.05 * i, 0.0] for i in range(n_kf)])
    fwd = np.array([0.0, 1.0, 0.0])
    kf_true = np.array([_pose_looking(c, fwd + np.array([0.05 * i, 0, 0]))
                        for i, c in enumerate(centres)])
    lms, obs = [], []
    for i in range(n_kf - 1):
        lms.append(np.array([0.3 * i + 0.15, 4.0 + 0.5 * i, 0.2 * (-1) ** i]))
        obs.append([i, i + 1])
    for i in range(n_kf):
        for q in range(leaves_per_kf):
            d = rng.uniform(3.0, 6.0)
            lms.append(centres[i] + np.array([rng.uniform(-1, 1), d,
                                              rng.uniform(-0.8, 0.8)]))
            obs.append([i])
    lm_true = np.array(lms)
    for o, l in zip(obs, lm_true):
        vis = _visible(cam, _camera_points(kf_true[o], l[None]))[0]
        assert vis.all(), "tree fixture landmark not visible"
    return _assemble("tree_chain", cam, kf_true, lm_true, obs, rng, 0.0,
                     0.02, 0.02, 0.05)


def make_star(n_lm: int = 6, seed: int = 6, sigma: float = 1.0) -> BAProblem:
    """Star tree: one anchored keyframe and n_lm landmarks seen once each,
    plus a second keyframe joined through a single landmark."""
    return make_tree_chain(2, leaves_per_kf=n_lm // 2, seed=seed, sigma=sigma)


def concat_problems(problems) -> dict:
    """Index offsets of a block-diagonal concatenation of problems."""
    kf_off = np.cumsum([0] + [p.n_keyframes for p in problems])
    lm_off = np.cumsum([0] + [p.n_landmarks for p in problems])
    f_off = np.cumsum([0] + [p.n_factors for p in problems])
    return dict(kf_off=kf_off, lm_off=lm_off, f_off=f_off)


# ----------------------------------------------------------------------------
# incremental stream (keyframes and landmarks arriving over time)
# ----------------------------------------------------------------------------

@dataclass
class IncrementalStream:
    """A full problem plus the order in which its parts arrive.

    `base` is the starting problem (the first n0 keyframes and the landmarks
    they spawn). Each element of `steps` adds one keyframe (initialised at
    the previous keyframe's current estimate by the caller), a block of new
    landmarks with initial positions, and the new measurement factors."""
    full: BAProblem
    base: BAProblem
    steps: list


def make_incremental_stream(seed: int = 20000, n_kf: int = 300, n0: int = 5,
                            new_lm_per_kf: int = 15, obs_range=(3, 8),
                            init_depth: float | None = 1.0,
                            sigma: float = 1.0) -> IncrementalStream:
    """Incremental SLAM stream along a random walk. Every landmark is spawned
    by one keyframe and observed by that keyframe and up to a few of the
    keyframes before it that also see it (triangulated at arrival). A new
    landmark is initialised along the spawning keyframe's ray at
    `init_depth` metres (the SLAM protocol of Section 9.2), or with N(0,0.1m)
    noise when init_depth is None."""
    rng = np.random.default_rng(seed)
    cam = Camera(sigma=sigma)
    centres, heading = _walk(n_kf, rng)
    kf_true = np.array([_pose_looking(c, np.array([np.cos(h), np.sin(h), 0.0]))
                        for c, h in zip(centres, heading)])
    rots = _rotmat(kf_true[:, :3])
    lms, obs, spawn = [], [], []
    per_kf = [new_lm_per_kf * 4 if k < n0 else new_lm_per_kf for k in range(n_kf)]
    for k in range(n_kf):
        made = 0
        while made < per_kf[k]:
            u = rng.uniform(40, cam.width - 40)
            v = rng.uniform(40, cam.height - 40)
            d = rng.uniform(2.0, 8.0)
            pc = np.array([(u - cam.cx) / cam.fx * d, (v - cam.cy) / cam.fy * d, d])
            pw = rots[k].T @ (pc - kf_true[k, 3:])
            prev = np.arange(max(0, k - 12), k)
            vis = prev[_visible(cam, _camera_points(kf_true[prev], pw[None]))[0]] \
                if len(prev) else prev
            want = int(rng.integers(obs_range[0], obs_range[1] + 1)) - 1
            if k >= 1 and len(vis) < 1:
                continue
            chosen = np.sort(rng.choice(vis, min(want, len(vis)), replace=False)) \
                if len(vis) else np.zeros(0, dtype=int)
            lms.append(pw)
            obs.append(np.concatenate([chosen, [k]]).astype(np.int32))
            spawn.append(k)
            made += 1
    lm_true = np.array(lms)
    full = _assemble("incremental", cam, kf_true, lm_true, obs, rng, 0.0,
                     0.05, 0.05, 0.1)
    spawn = np.array(spawn)
    if init_depth is not None:
        # depth init_depth along the spawning keyframe's measured ray
        for j in range(len(lm_true)):
            k = spawn[j]
            zf = full.z[_first_factor(full, j, k)]
            ray = np.array([(zf[0] - cam.cx) / cam.fx, (zf[1] - cam.cy) / cam.fy, 1.0])
            full.lm_init[j] = rots[k].T @ (init_depth * ray - kf_true[k, 3:])
    base_lm = np.flatnonzero(spawn < n0)
    base_f = np.flatnonzero(np.isin(full.factor_lm, base_lm))
    remap = -np.ones(len(lm_true), dtype=np.int64)
    remap[base_lm] = np.arange(len(base_lm))
    base = BAProblem("incremental_base", cam, kf_true[:n0], lm_true[base_lm],
                     full.kf_init[:n0], full.lm_init[base_lm],
                     full.factor_kf[base_f], remap[full.factor_lm[base_f]].astype(np.int32),
                     full.z[base_f], full.z_true[base_f], full.inlier[base_f],
                     full.kf_anchor_info[:n0])
    steps = []
    for k in range(n0, n_kf):
        new_lm = np.flatnonzero(spawn == k)
        new_f = np.flatnonzero(spawn[full.factor_lm] == k)
        steps.append(dict(kf=k, lm=new_lm, factors=new_f))
    return IncrementalStream(full, base, steps)


def _first_factor(p: BAProblem, j: int, k: int) -> int:
    idx = np.flatnonzero((p.factor_lm == j) & (p.factor_kf == k))
    return int(idx[0])


def reinit_at_depth(p: BAProblem, depth: float = 1.0) -> BAProblem:
    """A copy of `p` whose landmarks start `depth` metres along the measured
    ray of their newest observing keyframe, placed with that keyframe's
    initial pose (the monocular SLAM initialisation of Section 9.2)."""
    q = BAProblem(p.name + f"_depth{depth:g}", p.cam, p.kf_true, p.lm_true, p.kf_init.copy(),
                  p.lm_init.copy(), p.factor_kf, p.factor_lm, p.z, p.z_true, p.inlier, p.kf_anchor_info)
    cam = p.cam
    rots = _rotmat(p.kf_init[:, :3])
    for j in range(p.n_landmarks):
        fs = np.flatnonzero(p.factor_lm == j)
        if fs.size == 0:
            continue
        f = fs[np.argmax(p.factor_kf[fs])]
        k = int(p.factor_kf[f])
        ray = np.array([(p.z[f, 0] - cam.cx) / cam.fx, (p.z[f, 1] - cam.cy) / cam.fy, 1.0])
        q.lm_init[j] = rots[k].T @ (depth * ray - p.kf_init[k, 3:])
    return q
