"""Per-scene choice of the tile-group side (the group-size study of the paper's sensitivity
analysis, made a run-time decision).

Which group side renders a scene fastest depends on the scene and the resolution: grouping
shrinks the sort by the load reduction but adds staging work per member tile, and where the
balance falls differs from the paper's hardware (on the sensitivity workloads here 4x4 groups
win at 3M Gaussians, 8x8 groups in the dense 6M scene).  With the MFMA precisions every group
side, with or without opacity-aware culling, gives the same image (bit-identical with per-tile
rows), so the choice changes only the speed: `AdaptiveRenderer` renders the first frames of a
scene with each candidate (group side, culling) variant, timed on the stream with HIP events,
and then keeps the fastest (re-probing after `reprobe_every` frames, or after
`chooser.reset()`).  By default each probe frame renders its view with every variant, so the
variants are compared on the same views.
"""
from __future__ import annotations

from typing import Dict, Iterable, Optional

from . import gs


class GroupChooser:
    """Probe-then-commit policy: each candidate is tried `probes` times (round robin), then
    the one with the lowest best time is used until the next re-probe (the best of its probes,
    so a first frame that also grew the entry buffers does not count against a side)."""

    def __init__(self, candidates: Iterable[int], probes: int = 2, reprobe_every: int = 0):
        self.candidates = list(candidates)
        if not self.candidates:
            raise ValueError("no candidate group sides")
        self.probes = max(1, int(probes))
        self.reprobe_every = int(reprobe_every)
        self.reset()

    def reset(self):
        self.times: Dict[int, list] = {g: [] for g in self.candidates}
        self.chosen: Optional[int] = None
        self.since = 0

    def next(self) -> int:
        """The group side to render the next frame with."""
        if self.chosen is not None:
            if self.reprobe_every and self.since >= self.reprobe_every:
                self.reset()
            else:
                return self.chosen
        # round robin: the candidate probed least so far (first in order on ties)
        g = min(self.candidates, key=lambda c: len(self.times[c]))
        return g if len(self.times[g]) < self.probes else self._commit()

    def observe(self, group: int, ms: float):
        if self.chosen is None:
            self.times[group].append(float(ms))
            if all(len(t) >= self.probes for t in self.times.values()):
                self._commit()
        else:
            self.since += 1

    def _commit(self) -> int:
        self.chosen = min(self.candidates, key=lambda g: (min(self.times[g]), g))
        self.since = 0
        return self.chosen


class AdaptiveRenderer:
    """Renders frames of one scene with the (group side, culling) variant a GroupChooser picks;
    one gs.Renderer (and its buffers) per group side."""

    def __init__(self, n: int, width: int, height: int, precision="fp16", splits: int = 2,
                 groups=(1, 2, 4, 8), tight=(False, True), probes: int = 2, reprobe_every: int = 0,
                 bg=(0.0, 0.0, 0.0), device="cuda", tile_rows: bool = False, paired: bool = True):
        prec = gs.PRECISIONS[precision] if isinstance(precision, str) else precision
        if prec == gs.GS_PREC_FP32:
            groups = [g for g in groups if g != 8]      # the FP32 rasterizer has no 8x8 groups
        tights = (tight,) if isinstance(tight, bool) else tuple(tight)
        self.n, self.width, self.height = n, width, height
        self.variants = [(g, t) for g in groups for t in tights]
        # tile_rows: grouped MFMA variants build rows per member tile, so every variant's image is
        # bit-identical to the 1x1 one; by default they build them once per group (same image to
        # the 16-bit operands' rounding)
        self.opts = {v: gs.options(group=v[0], precision=prec, splits=splits, bg=bg, tight=v[1], tile_rows=tile_rows)
                     for v in self.variants}
        self.renderers = {g: gs.Renderer(n, width, height, group=g, device=device) for g in groups}
        self.chooser = GroupChooser(self.variants, probes, reprobe_every)
        # paired: a probe frame renders its view with every variant (one probe round), instead of
        # one variant per frame in turn, whose views differ from variant to variant
        self.paired = paired
        self.last_variant = None

    def _timed(self, scene, cam, v, st) -> float:
        import torch
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        self.renderers[v[0]].render(scene, cam, self.opts[v], stream=st)
        b.record(st)
        b.synchronize()
        return a.elapsed_time(b)

    def render(self, scene: "gs.DeviceScene", cam, stream=None):
        """Renders one frame; returns (image tensor, (group side, culling) used)."""
        import torch
        if (cam.width, cam.height) != (self.width, self.height):
            raise ValueError("camera size differs from the renderer's")
        v = self.chooser.next()
        st = stream if stream is not None else torch.cuda.current_stream()
        if self.chooser.chosen is None and self.paired:
            # one probe round on this view; the image returned is the last variant's
            for v in self.variants:
                self.chooser.observe(v, self._timed(scene, cam, v, st))
            self.last_variant = v
            return self.renderers[v[0]].image, v
        ren = self.renderers[v[0]]
        if self.chooser.chosen is None:
            self.chooser.observe(v, self._timed(scene, cam, v, st))
        else:
            ren.render(scene, cam, self.opts[v], stream=st)
            self.chooser.observe(v, 0.0)
        self.last_variant = v
        return ren.image, v
