"""Sections of keyframes around the splat [Sec. 3.2-3.5]: the visibility
check and the overlap-section selection with batched pre-tracking (Sec. 3.3),
complement initialisation of uncovered pixels (Sec. 3.4) and the section
lifecycle -- one learnable section resident, finished sections frozen and
kept in host memory until a head frame needs one as its overlapping section.

Host-side orchestration only: every per-pixel step runs in the HIP library
(``vtgs_visibility``, ``vtgs_uncovered_mask``, ingestion, ``track_step``).
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import check, load
from .render import Camera, Keyframe, Plan, View, _dev, _ptr, _stream, track_cfg


def frame_ref(depth_map, cam, pose):
    """A vtgs_frame_ref of a device depth map [H*W], a camera and a device
    pose [12]."""
    return _lib.vtgs_frame_ref(_ptr(depth_map), Camera.of(cam).cstruct(), _ptr(pose))


def keyframe_ref(k: Keyframe):
    """The frame a keyframe was ingested from (its depth map and pose)."""
    if k.depth_map is None:
        raise ValueError("keyframe has no depth map (ingest it with Keyframe.ingest)")
    return frame_ref(k.depth_map, k.cam, k.pose)


def visibility(src_depth, src_cam, src_pose, targets, rel_tol=0.01, z_near=0.01, want_mask=True,
               want_counts=True, stream=None):
    """Sec. 3.3 visibility check: for each valid source pixel, whether its
    point lies within rel_tol of a target's interpolated depth.  targets:
    vtgs_frame_ref list.  Returns (mask uint8 [H*W] union over the targets or
    None, counts int32 [n_targets] or None), on the device."""
    L = load()
    dev = src_depth.device
    cam = Camera.of(src_cam)
    mask = torch.empty(cam.P, dtype=torch.uint8, device=dev) if want_mask else None
    counts = torch.empty(len(targets), dtype=torch.int32, device=dev) if want_counts else None
    tg = (_lib.vtgs_frame_ref * len(targets))(*targets)
    sc = cam.cstruct()
    check(L.vtgs_visibility(_ptr(src_depth), C.byref(sc), _ptr(src_pose), tg, len(targets),
                            float(rel_tol), float(z_near), _ptr(mask), _ptr(counts),
                            _stream(stream)))
    return mask, counts


def section_mask(src_depth, src_cam, src_pose, section, rel_tol=0.01, stream=None):
    """Eq. 1's visibility mask W of a frame against a section (Sec. 3.3):
    the union of its visibility in the section's head, middle and last
    keyframes."""
    ks = section.keyframes
    picks = sorted({0, len(ks) // 2, len(ks) - 1})
    mask, _ = visibility(src_depth, src_cam, src_pose, [keyframe_ref(ks[i]) for i in picks],
                         rel_tol, want_counts=False, stream=stream)
    return mask


def select_overlap(counts, n_valid, candidate_sections, gamma, n_front=3):
    """First stage of the overlapping-section selection (Sec. 3.3): keep the
    candidate views whose count of visible points exceeds gamma times the
    frame's valid points, then the n_front most front (earliest) sections
    that hold one of them, each once."""
    chosen = set()
    for c, s in zip(counts, candidate_sections):
        if c > gamma * n_valid:
            chosen.add(int(s))
    return sorted(chosen)[:n_front]


class Section:
    """Consecutive keyframes mapped together (Sec. 3.2); index = position in
    the sequence (smaller = more front)."""

    def __init__(self, index, keyframes):
        self.index = int(index)
        self.keyframes = list(keyframes)
        self.frozen = False
        self.host = None  # host copies while offloaded

    @property
    def n_gaussians(self):
        return sum(k.n for k in self.keyframes)

    @property
    def resident(self):
        return self.host is None


def overlap_candidates(sections, n1=5):
    """Candidate views for the overlap selection: every n1-th keyframe of the
    earlier sections (App. A: N1 = 5), with its section index."""
    out = []
    j = 0
    for s in sections:
        for k in s.keyframes:
            if j % n1 == 0:
                out.append((s.index, k))
            j += 1
    return out


def pretrack(sections, cam, init_pose, obs_rgb, obs_depth, iters=10, cfg=None, masks=None,
             prm=None, device=None, stream=None):
    """Pre-tracking of one head frame against each candidate section
    (Sec. 3.3), all in one batched track plan: view v renders section v's
    keyframes from its own copy of the initial pose with its own Adam state
    and visibility mask.  Returns (index of the section with the smallest
    final Eq. 1 loss, losses [iters, n_sections] on the host, the views)."""
    dev = _dev(device)
    kfs, views = [], []
    for i, s in enumerate(sections):
        first = len(kfs)
        kfs.extend(s.keyframes)
        vis = None if masks is None else masks[i]
        views.append(View(cam, torch.as_tensor(init_pose, dtype=torch.float32, device=dev)
                          .reshape(12).clone(), first, len(s.keyframes), obs_rgb, obs_depth, vis,
                          device=dev).with_pose_adam())
    plan = Plan(kfs, views, prm, device=dev, stream=stream)
    loss = plan.track_step(cfg if cfg is not None else track_cfg(), iters=iters, stream=stream)
    rc, need = plan.status(stream=stream)
    if rc != _lib.VTGS_OK:
        raise _lib.VtgsError(rc, _lib.last_error())
    L = loss.cpu()
    best = int(torch.argmin(L[-1]).item())
    return best, L, views


def choose_overlap_section(head_depth, head_rgb, cam, init_pose, sections, gamma, n1=5,
                           n_front=3, iters=10, cfg=None, prm=None, stream=None):
    """The whole overlapping-section selection for a head frame (Sec. 3.3):
    candidate views every n1 keyframes, visibility counts from the initial
    pose, the n_front most front sections above gamma, batched pre-tracking
    with each section's visibility mask, the smallest loss wins.  Returns
    (chosen Section or None, its refined pose [12], details)."""
    dev = head_depth.device
    pose = torch.as_tensor(init_pose, dtype=torch.float32, device=dev).reshape(12).contiguous()
    cands = overlap_candidates(sections, n1)
    if not cands:
        return None, pose, {}
    _, counts = visibility(head_depth, cam, pose, [keyframe_ref(k) for _, k in cands],
                           want_mask=False, stream=stream)
    n_valid = int((head_depth > 0).sum().item())
    picked = select_overlap(counts.cpu().tolist(), n_valid, [s for s, _ in cands], gamma, n_front)
    if not picked:
        return None, pose, dict(counts=counts.cpu(), n_valid=n_valid, picked=[])
    by_index = {s.index: s for s in sections}
    secs = [by_index[i] for i in picked]
    masks = [section_mask(head_depth, cam, pose, s, stream=stream) for s in secs]
    best, losses, views = pretrack(secs, cam, pose, head_rgb, head_depth, iters, cfg, masks, prm,
                                   dev, stream)
    return secs[best], views[best].pose, dict(counts=counts.cpu(), n_valid=n_valid, picked=picked,
                                              losses=losses, masks=masks)


# ----------------------------------------------------------------------------
# complement initialisation and the section lifecycle (Sec. 3.2, 3.4)
# ----------------------------------------------------------------------------

def uncovered_mask(sil, depth_map, thr=0.5, stream=None):
    """Pixels a frame's current rendering leaves uncovered (silhouette below
    thr, Sec. 3.4 / App. A 0.5) that hold a valid depth: uint8 [P]."""
    n = depth_map.numel()
    mask = torch.empty(n, dtype=torch.uint8, device=depth_map.device)
    check(load().vtgs_uncovered_mask(_ptr(sil), _ptr(depth_map), n, float(thr), _ptr(mask),
                                     _stream(stream)))
    return mask


def complement_keyframe(section, depth_img, rgb_img, cam, pose, thr=0.5, o_init=0.99, prm=None,
                        stream=None):
    """Sec. 3.4: render the section's Gaussians at a regular frame's pose and
    tie new Gaussians to the pixels they leave uncovered.  Returns the new
    (learnable) keyframe, or None when every valid pixel is covered, and the
    mask."""
    dev = section.keyframes[0].depth.device
    cam = Camera.of(cam)
    d = torch.as_tensor(depth_img, dtype=torch.float32).to(dev).reshape(-1).contiguous()
    pose_t = torch.as_tensor(pose, dtype=torch.float32).to(dev).reshape(12).contiguous()
    plan = Plan(section.keyframes, [View(cam, pose_t, 0, len(section.keyframes), device=dev)], prm,
                device=dev, stream=stream)
    _, _, sil = plan.render_fwd(stream=stream)
    rc, _ = plan.status(stream=stream)
    if rc != _lib.VTGS_OK:
        raise _lib.VtgsError(rc, _lib.last_error())
    mask = uncovered_mask(sil, d, thr, stream)
    if int(mask.sum().item()) == 0:
        return None, mask
    k = Keyframe.ingest(d.reshape(cam.height, cam.width), rgb_img, cam, pose_t, 1, o_init,
                        mask.reshape(cam.height, cam.width), True, dev, stream)
    return k, mask


_KF_TENSORS = ("pix", "depth", "color", "opacity", "radius", "pose", "depth_map")


class SectionStore:
    """The sections of one sequence (Sec. 3.2): the current section is
    learnable and resident; a finished one is frozen (no more gradients) and
    may be offloaded to pinned host memory, from where it is prefetched when
    a head frame renders it as its overlapping section S^o (Sec. 3.3).  Keeps
    the counts of Tab. 9: Gaussians created in total and the most resident
    at a time.  Copies run on their own stream (default priority); a
    prefetch returns an event the rendering stream waits on.  Offloading
    replaces a keyframe's tensors, so plans over a section are built after
    its prefetch, never kept across an offload."""

    def __init__(self, device=None):
        self.device = _dev(device)
        self.sections = []
        self.total_gaussians = 0
        self.peak_resident = 0
        self._copy = torch.cuda.Stream(self.device) if self.device.type == "cuda" else None

    @property
    def current(self):
        return self.sections[-1] if self.sections else None

    def resident_gaussians(self):
        return sum(s.n_gaussians for s in self.sections if s.resident)

    def _account(self):
        self.peak_resident = max(self.peak_resident, self.resident_gaussians())

    def start_section(self, head: Keyframe) -> Section:
        """A head frame starts a new section; the previous one is frozen."""
        if self.current is not None:
            self.freeze(self.current)
        s = Section(len(self.sections), [head])
        self.sections.append(s)
        self.total_gaussians += head.n
        self._account()
        return s

    def add_keyframe(self, k: Keyframe):
        """A complement keyframe of a regular frame joins the current section."""
        self.current.keyframes.append(k)
        self.total_gaussians += k.n
        self._account()

    def freeze(self, s: Section):
        """No more learning for s: its keyframes drop gradient and optimiser
        state (plans built afterwards treat them as fixed)."""
        for k in s.keyframes:
            k.learnable = False
            k.g_color = k.g_opacity = k.g_radius = k.adam = None
            k.g_depth = k.g_pose = k.depth_adam = k.pose_adam = None
        s.frozen = True

    def offload(self, s: Section):
        """Move a frozen section to pinned host memory (asynchronous on the
        copy stream; the device memory returns to the allocator once the
        copies are done)."""
        if not s.frozen:
            raise ValueError("only a frozen section is offloaded")
        if not s.resident:
            return
        pin = self.device.type == "cuda"
        host = []
        cur = torch.cuda.current_stream(self.device) if pin else None
        if pin:
            self._copy.wait_stream(cur)
        for k in s.keyframes:
            h = {}
            for name in _KF_TENSORS:
                t = getattr(k, name)
                if t is None:
                    continue
                dst = torch.empty(t.shape, dtype=t.dtype, pin_memory=pin)
                if pin:
                    with torch.cuda.stream(self._copy):
                        dst.copy_(t, non_blocking=True)
                    t.record_stream(self._copy)
                else:
                    dst.copy_(t)
                h[name] = dst
                setattr(k, name, None)
            host.append(h)
        if pin:
            ev = torch.cuda.Event()
            ev.record(self._copy)
            ev.synchronize()  # host copies complete before they are read
        s.host = host

    def prefetch(self, s: Section):
        """Bring an offloaded section back to the device on the copy stream;
        returns an event the rendering stream waits on (None if resident)."""
        if s.resident:
            return None
        pin = self.device.type == "cuda"
        cur = torch.cuda.current_stream(self.device) if pin else None
        if pin:
            self._copy.wait_stream(cur)
        for k, h in zip(s.keyframes, s.host):
            for name, src in h.items():
                if pin:
                    with torch.cuda.stream(self._copy):
                        dst = src.to(self.device, non_blocking=True)
                    dst.record_stream(cur)  # used (and freed) on the rendering stream
                else:
                    dst = src.clone()
                setattr(k, name, dst)
        s.host = None
        self._account()
        if pin:
            ev = torch.cuda.Event()
            ev.record(self._copy)
            return ev
        return None


# -- checkpoint / resume ---------------------------------------------------------
# The map is plain tensors: per keyframe its pixel indices, tied depths,
# colour, opacity, radius, pose (and depth map), the learnable section's
# optimiser states, and the sections' structure.  A checkpoint is one
# safetensors file (tensors only, nothing executable) whose metadata holds
# the structure as JSON.
_KF_STATE = ("adam", "depth_adam", "pose_adam")


def save_map(store: SectionStore, path):
    """Write the store's sections (resident or offloaded) to `path`."""
    import json
    from safetensors.torch import save_file
    tensors, sections = {}, []
    for s in store.sections:
        kfs = []
        host = s.host if not s.resident else None
        for j, k in enumerate(s.keyframes):
            tag = "s%d.k%d." % (s.index, j)
            for name in _KF_TENSORS + _KF_STATE:
                t = host[j].get(name) if host is not None and name in _KF_TENSORS else getattr(k, name)
                if t is not None:
                    tensors[tag + name] = t.detach().to("cpu").contiguous()
            c = k.cam
            kfs.append(dict(cam=[c.fx, c.fy, c.cx, c.cy, c.width, c.height], learnable=k.learnable))
        sections.append(dict(index=s.index, frozen=s.frozen, offloaded=not s.resident, keyframes=kfs))
    meta = dict(sections=json.dumps(sections), total_gaussians=str(store.total_gaussians),
                peak_resident=str(store.peak_resident))
    save_file(tensors, str(path), metadata=meta)


def load_map(path, device=None) -> SectionStore:
    """A store rebuilt from `save_map`'s file: every section resident on
    `device` (offloaded ones come back frozen), the learnable section with
    its gradient buffers and optimiser states."""
    import json
    from safetensors import safe_open
    dev = _dev(device)
    store = SectionStore(dev)
    with safe_open(str(path), framework="pt", device="cpu") as f:
        meta = f.metadata()
        names = set(f.keys())
        for sd in json.loads(meta["sections"]):
            kfs = []
            for j, kd in enumerate(sd["keyframes"]):
                tag = "s%d.k%d." % (sd["index"], j)
                get = lambda n: f.get_tensor(tag + n).to(dev) if tag + n in names else None
                k = Keyframe(tuple(kd["cam"]), get("pose"), get("pix"), get("depth"), get("color"),
                             get("opacity"), get("radius"), learnable=kd["learnable"], device=dev)
                k.depth_map = get("depth_map")
                if k.learnable:
                    k.with_grad_buffers()
                    for n in _KF_STATE:
                        setattr(k, n, get(n))
                    if k.depth_adam is not None or k.pose_adam is not None:
                        k.with_geometry_grads()
                kfs.append(k)
            s = Section(sd["index"], kfs)
            s.frozen = bool(sd["frozen"])
            store.sections.append(s)
        store.total_gaussians = int(meta["total_gaussians"])
        store.peak_resident = int(meta["peak_resident"])
    return store
