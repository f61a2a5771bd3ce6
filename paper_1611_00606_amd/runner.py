"""Device-resident build of one problem: uploads inputs once, owns H, S, the
workspace and the info flags, and enqueues hs_build_ex on demand.

Marshalling only: the build itself runs in the HIP library.
"""

from __future__ import annotations

import numpy as np

from ._binding import HS_FP64, hs_build_ex, hs_workspace_bytes


class DeviceBuild:
    def __init__(self, A, B, T_AA, T_AB, T_BB, U, nl, n_g, device="cuda:0", mode=HS_FP64,
                 batch=0, tuning=None):
        import torch
        self.device = torch.device(device)
        nl = np.asarray(nl, dtype=np.int32)
        self.N_A = int(nl.shape[0])
        self.N_G = int(n_g)
        self.uniform = bool(np.all(nl == nl[0]))
        self.N_L = int(nl[0]) if self.uniform else int(nl.max())
        self.nl_per_atom = None if self.uniform else nl
        self.mode = mode
        self.batch = int(batch)
        self.tuning = tuning

        def up(x):
            return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to(self.device)

        self.A, self.B = up(A), up(B)
        self.T_AA, self.T_AB, self.T_BB, self.U = up(T_AA), up(T_AB), up(T_BB), up(U)
        self.H = torch.empty((self.N_G, self.N_G), dtype=torch.complex128, device=self.device)
        self.S = torch.empty_like(self.H)
        self.info = torch.empty(self.N_A, dtype=torch.int32, device=self.device)
        nbytes = hs_workspace_bytes(self.N_A, self.nl_per_atom, self.N_L, self.N_G, mode)
        if nbytes == 0:
            raise ValueError("invalid problem size")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    @classmethod
    def from_problem(cls, p, device="cuda:0", **kw):
        return cls(p.A, p.B, p.T_AA, p.T_AB, p.T_BB, p.U, p.nl, p.N_G, device=device, **kw)

    def run(self, stream=None, phase_events=None):
        """Enqueue one build on `stream` (default: the current stream)."""
        return hs_build_ex(self.A, self.B, self.T_AA, self.T_AB, self.T_BB, self.U,
                           self.N_A, self.N_L, self.N_G, self.H, self.S,
                           workspace=self.workspace, info=self.info, stream=stream,
                           mode=self.mode, nl_per_atom=self.nl_per_atom,
                           phase_events=phase_events, batch=self.batch, tuning=self.tuning)

    def results(self):
        """(H, S, info) as host numpy arrays (synchronizes)."""
        return self.H.cpu().numpy(), self.S.cpu().numpy(), self.info.cpu().numpy()
