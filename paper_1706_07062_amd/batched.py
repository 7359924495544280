"""Many images (or particle sets) of uneven size in one persistent launch.

All rays of all images live in one structure-of-arrays state; one init launch
fills it from the camera table and one persistent integrate launch works
through it with XCD-partitioned work stealing, so images of 32^2 and 1024^2
rays, and rays of 20 and 2,000 steps, share the machine without per-image
tails.  The launch shape comes from the autotuner, and the sequence
init -> integrate -> device statistics is captured once into a HIP graph and
replayed.
"""
from __future__ import annotations

import torch

from . import Context, State, autotune, kh_camera


def camera_struct(cam) -> kh_camera:
    return kh_camera(cam.a, cam.r_obs, cam.incl, cam.alpha_min, cam.alpha_max, cam.beta_min, cam.beta_max,
                     cam.width, cam.height)


class BatchedImages:
    def __init__(self, ctx: Context, cams, params, k_cross: int = 0, constants: bool = True, tune: bool = True,
                 tune_stride: int = 16, tune_key: str = "batched", log=None):
        self.ctx = ctx
        self.cams = list(cams)
        self.kcams = [camera_struct(c) for c in self.cams]
        self.n = sum(c.width * c.height for c in self.cams)
        self.state = State(self.n, k_cross=k_cross, constants=constants)
        self.stats_dev = torch.zeros(8, dtype=torch.int64, device="cuda")
        self.params = params
        self.choice = {}
        if tune:
            self.choice = self._tune(tune_stride, tune_key, k_cross, log)
            self.params = autotune.apply(params, self.choice)
        # upload the camera table once; later inits reuse it (graph-capturable)
        self.ctx.kh_init_rays(self.kcams, self.state)
        torch.cuda.synchronize()
        self.graph = None

    def _tune(self, stride, key, k_cross, log):
        """Tune on every `stride`-th image, in a context of its own so the main
        context's camera table is untouched."""
        sub = self.kcams[::stride]
        n_sub = sum(c.width * c.height for c in sub)
        tctx = Context(self.ctx.device)
        st = State(n_sub, k_cross=k_cross, constants=False)
        tctx.kh_init_rays(sub, st)

        def reinit():
            tctx.kh_init_rays(None, st, n_cams=len(sub))

        choice = autotune.tune(tctx, reinit, st, self.params, key=f"{key}|n{n_sub}", log=log)
        tctx.close()
        return choice

    def run_eager(self, stream=None):
        self.ctx.kh_init_rays(None, self.state, n_cams=len(self.kcams), stream=stream)
        self.ctx.kh_integrate(self.params, self.state, stream=stream)
        self.ctx.kh_stats_device(self.state, self.stats_dev, stream=stream)

    def capture(self):
        """Capture init -> integrate -> statistics into a HIP graph."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.run_eager(stream=side)  # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run_eager()
        torch.cuda.synchronize()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()

    def stats(self) -> dict:
        v = self.stats_dev.cpu().tolist()
        return dict(status_counts=v[:6], n_acc=v[6], n_rej=v[7])
