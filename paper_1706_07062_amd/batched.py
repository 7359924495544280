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


class ImageStream:
    """Frames of images (each a list of cameras with the same total ray count)
    integrated back to back, with the copy of each frame's final states to
    host memory overlapping the integration of the next: two device states
    used in turn, two page-locked host buffers, a compute stream and a copy
    stream with a context each (a context is not shared between streams that
    run at the same time).  `consume(frame_index, states, statuses)` gets the
    host rows ([n][8] float64 and [n] int32 CPU tensors) of each frame in
    order; they are overwritten two frames later, so it copies what it keeps.
    The overlap needs the two streams on different hardware queues; the
    runtime spreads streams over a few queues (four by default), so create
    the stream before a program has made many others."""

    def __init__(self, device: int, n: int, params, k_cross: int = 0):
        self.n = n
        self.params = params
        self.cctx = Context(device)
        self.xctx = Context(device)
        self.sc = torch.cuda.Stream(device=device)
        self.sx = torch.cuda.Stream(device=device)
        self.states = [State(n, k_cross=k_cross, constants=False) for _ in range(2)]
        self.host = [(torch.empty((n, 8), dtype=torch.float64, pin_memory=True),
                      torch.empty(n, dtype=torch.int32, pin_memory=True)) for _ in range(2)]
        self.done = [torch.cuda.Event() for _ in range(2)]
        torch.cuda.synchronize()

    def run(self, frames, consume):
        def read(f):
            b = f % 2
            self.sx.wait_event(self.done[b])
            # synchronous on the copy stream: the host rows are complete on return
            self.xctx.kh_read_state(self.states[b], out=self.host[b], stream=self.sx)
            consume(f, *self.host[b])

        count = 0
        for f, cams in enumerate(frames):
            kc = [camera_struct(c) for c in cams]
            if sum(c.width * c.height for c in cams) != self.n:
                raise ValueError(f"frame {f} does not have {self.n} rays")
            b = f % 2
            # state b was last read back (synchronously) for frame f - 2
            self.cctx.kh_init_rays(kc, self.states[b], stream=self.sc)
            self.cctx.kh_integrate(self.params, self.states[b], stream=self.sc)
            self.done[b].record(self.sc)
            if f >= 1:
                read(f - 1)
            count = f + 1
        if count:
            read(count - 1)
        torch.cuda.synchronize()
        return count

    def close(self):
        self.cctx.close()
        self.xctx.close()
