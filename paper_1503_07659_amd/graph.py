"""Capture library launches in a HIP graph (through torch's graph API).

The library's launches take everything by value (pointers, sizes, the group
table) and need no device-side state, so a captured launch replays exactly.
Before capture, the launch runs once on a side stream so that the library's
per-device queries (CU count, occupancy, LDS limit) are cached and no setup
call happens inside the capture.  Nothing in the captured work clears memory
(no memset nodes).
"""

import torch


class CapturedLaunch:
    """Capture `fn()` (which launches library kernels on the current stream) once; replay() reruns it."""

    def __init__(self, fn, warmup=1):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            fn()
        torch.cuda.synchronize()

    def replay(self):
        self.graph.replay()
