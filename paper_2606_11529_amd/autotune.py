"""Autotuner for the launch knobs of the hot path.

Like the paper's hyperparameter selection (Methodology section, the phased
search that profiles the views to be rendered once and reuses the result for
that scene on that hardware), it renders the target views and searches, in
phases:
  1. tile size (8x8 or 16x16; this changes the pair lists, so the sort is
     re-profiled per tile size) and sort strategy (presort / full);
  2. forward compositing: LDS batch x pixels per thread;
  3. backward compositing: LDS batch x pixels per thread;
  4. tile schedule: tiles in index order, longest list first, or longest
     first on a persistent grid (the analogue of the paper's trip-count
     binning), timed as binning + forward + backward since the order is
     built during binning.
None of these knobs changes the rendered image except the tile size (the
3-sigma rect is rounded out to whole tiles), which is only searched when the
caller allows it. Results are cached in JSON keyed by device, scene size, SH
degree and resolutions.
"""
from __future__ import annotations

import dataclasses
import json
import os
import statistics
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

LDS_BATCHES = (64, 128, 256, 512)
PPTS = (1, 2, 4)
SORTS = ("bands", "presort", "full")


def pick_best(timings: Dict[tuple, Sequence[float]], tie: float = 0.02) -> tuple:
    """Fastest candidate by median time; candidates within ``tie`` of the
    fastest are resolved towards the first one listed (the default order
    puts the safer/smaller configuration first)."""
    if not timings:
        raise ValueError("no timings")
    med = {k: statistics.median(v) for k, v in timings.items()}
    best = min(med.values())
    for k in timings:  # insertion order
        if med[k] <= best * (1.0 + tie):
            return k
    raise AssertionError


def cache_key(device: str, n: int, sh_degree: int, resolutions: Iterable[Tuple[int, int]],
              tiles: Iterable[int]) -> str:
    res = ",".join(f"{w}x{h}" for w, h in resolutions)
    return f"{device}|n={n}|sh={sh_degree}|res={res}|tiles={','.join(map(str, tiles))}"


def load_cache(path: Optional[str]) -> dict:
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(path: Optional[str], cache: dict) -> None:
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


@dataclasses.dataclass
class TuneResult:
    tile: int
    sort_mode: str
    fwd_lds: int
    fwd_ppt: int
    bwd_lds: int
    bwd_ppt: int
    ms: dict
    schedule: str = "index"  # "index" | "longest_first" | "persistent"

    def apply(self, cfg):
        """``cfg`` with the tuned knobs."""
        return dataclasses.replace(cfg, tile=self.tile, sort_mode=self.sort_mode,
                                   lds_batch=self.fwd_lds, fwd_ppt=self.fwd_ppt,
                                   bwd_lds_batch=self.bwd_lds, bwd_ppt=self.bwd_ppt,
                                   tile_order=self.schedule != "index",
                                   persistent=self.schedule == "persistent")


def _timer():
    import torch

    def time_call(fn: Callable[[], None], reps: int) -> List[float]:
        out = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            out.append(a.elapsed_time(b))
        return out
    return time_call


SCHEDULES = ("index", "longest_first", "persistent")


def autotune(scene, cams, cfg, tiles=(16,), lds_batches=LDS_BATCHES, ppts=PPTS, sorts=SORTS,
             reps: int = 3, cache_path: Optional[str] = None, verbose: bool = False,
             schedules: Sequence[str] = SCHEDULES) -> TuneResult:
    """Search the knobs on ``scene`` (a renderer.Scene) over ``cams``."""
    import torch

    from . import renderer as R

    dev = torch.cuda.get_device_name(scene.means.device)
    key = cache_key(dev, scene.n, cfg.sh_degree, [(c.width, c.height) for c in cams], tiles)
    cache = load_cache(cache_path)
    if key in cache:
        return TuneResult(**cache[key])
    time_call = _timer()
    ws = R.Workspace()
    ms = {}

    tile_rows = []
    for tile in tiles:
        c0 = dataclasses.replace(cfg, tile=tile)
        sort_t = {}
        states = []
        for sm in sorts:
            cs = dataclasses.replace(c0, sort_mode=sm)
            views = [R.Views([scene], [c], [0], cs) for c in cams]
            projs = [R.xpr_project(v, cs) for v in views]
            bins = [R.xpr_bin_sort(v, cs, p, ws=ws) for v, p in zip(views, projs)]

            def run_sort(cs=cs, views=views, projs=projs, bins=bins):
                for v, p, b in zip(views, projs, bins):
                    R.xpr_bin_sort(v, cs, p, capacity=b.capacity, ws=ws, out=b)
            run_sort()
            sort_t[sm] = time_call(run_sort, reps)
            states = [(v, p, b) for v, p, b in zip(views, projs, bins)]
        sm_best = pick_best(sort_t)
        ms[f"tile{tile}_sort"] = {k: statistics.median(v) for k, v in sort_t.items()}
        c1 = dataclasses.replace(c0, sort_mode=sm_best)
        frames = [R.xpr_render_fwd(v, c1, p, b) for v, p, b in states]
        fwd_t = {}
        for lds in lds_batches:
            for ppt in (ppts if tile == 16 else (1,)):
                cf = dataclasses.replace(c1, lds_batch=lds, fwd_ppt=ppt)
                vf = [R.Views([scene], [v.cams[0]], [0], cf) for v, _, _ in states]

                def run_fwd(cf=cf, vf=vf):
                    for v, (_, p, b), fr in zip(vf, states, frames):
                        R.xpr_render_fwd(v, cf, p, b, out=fr)
                run_fwd()
                fwd_t[(lds, ppt)] = time_call(run_fwd, reps)
        f_lds, f_ppt = pick_best(fwd_t)
        g2 = torch.empty((scene.n, 9), dtype=torch.float32, device=scene.means.device)
        dimgs = [torch.randn(3 * c.width * c.height, device=scene.means.device) * 1e-6
                 for c in cams]
        bwd_t = {}
        for lds in lds_batches:
            for ppt in (ppts if tile == 16 else (1,)):
                cb = dataclasses.replace(c1, bwd_lds_batch=lds, bwd_ppt=ppt)
                vb = [R.Views([scene], [v.cams[0]], [0], cb) for v, _, _ in states]

                def run_bwd(cb=cb, vb=vb):
                    for v, (_, p, b), fr, d in zip(vb, states, frames, dimgs):
                        R.xpr_render_bwd(v, cb, p, b, fr, d, params=False, grad2d=g2, ws=ws)
                run_bwd()
                bwd_t[(lds, ppt)] = time_call(run_bwd, reps)
        b_lds, b_ppt = pick_best(bwd_t)
        total = (statistics.median(sort_t[sm_best]) + statistics.median(fwd_t[(f_lds, f_ppt)]) +
                 statistics.median(bwd_t[(b_lds, b_ppt)]))
        ms[f"tile{tile}_fwd"] = {f"{k[0]}x{k[1]}": statistics.median(v) for k, v in fwd_t.items()}
        ms[f"tile{tile}_bwd"] = {f"{k[0]}x{k[1]}": statistics.median(v) for k, v in bwd_t.items()}
        tile_rows.append((total, tile, sm_best, f_lds, f_ppt, b_lds, b_ppt))
        if verbose:
            print(f"[autotune] tile {tile}: sort {sm_best}, fwd {f_lds}x{f_ppt}, "
                  f"bwd {b_lds}x{b_ppt}, {total:.3f} ms", flush=True)
    best = min(tile_rows)
    res = TuneResult(tile=best[1], sort_mode=best[2], fwd_lds=best[3], fwd_ppt=best[4],
                     bwd_lds=best[5], bwd_ppt=best[6], ms=ms)
    if len(schedules) == 1:
        res.schedule = schedules[0]
    else:
        res.schedule = _tune_schedule(scene, cams, res.apply(cfg), schedules, reps, time_call, ws,
                                      ms)
        if verbose:
            print(f"[autotune] schedule {res.schedule}", flush=True)
    cache[key] = dataclasses.asdict(res)
    save_cache(cache_path, cache)
    return res


def _tune_schedule(scene, cams, cfg, schedules, reps, time_call, ws, ms) -> str:
    """Phase 4: binning + forward + backward per tile schedule."""
    import torch

    from . import renderer as R

    g2 = torch.empty((scene.n, 9), dtype=torch.float32, device=scene.means.device)
    dimgs = [torch.randn(3 * c.width * c.height, device=scene.means.device) * 1e-6 for c in cams]
    t = {}
    for sch in schedules:
        cs = dataclasses.replace(cfg, tile_order=sch != "index", persistent=sch == "persistent")
        views = [R.Views([scene], [c], [0], cs) for c in cams]
        projs = [R.xpr_project(v, cs) for v in views]
        bins = [R.xpr_bin_sort(v, cs, p, ws=ws) for v, p in zip(views, projs)]
        frames = [R.xpr_render_fwd(v, cs, p, b) for v, p, b in zip(views, projs, bins)]

        def run(cs=cs, views=views, projs=projs, bins=bins, frames=frames):
            for v, p, b, fr, d in zip(views, projs, bins, frames, dimgs):
                R.xpr_bin_sort(v, cs, p, capacity=b.capacity, ws=ws, out=b)
                R.xpr_render_fwd(v, cs, p, b, out=fr)
                R.xpr_render_bwd(v, cs, p, b, fr, d, params=False, grad2d=g2, ws=ws)
        run()
        t[sch] = time_call(run, reps)
    ms["schedule"] = {k: statistics.median(v) for k, v in t.items()}
    return pick_best(t)
