"""Learned-match binding: mrf_mlp_* (create, synth, forward, grads, adam_step, train, match)."""
import ctypes

import numpy as np
import torch

from ._lib import MlpTrainCfg, check, lib
from .util import copy_from_ptr, copy_to_ptr, need, ptr, stream_ptr, workspace


class MLP:
    """n_in -> hidden x layers -> 2 ReLU network with library-owned FP32 parameters."""

    def __init__(self, n_in=20, hidden=256, layers=3, seed=0, device="cuda", stream=None):
        h = ctypes.c_void_p()
        check(lib.mrf_mlp_create(int(n_in), int(hidden), int(layers), 2, ctypes.c_uint64(seed), stream_ptr(stream),
                                 ctypes.byref(h)), "mrf_mlp_create")
        self.handle = h
        self.n_in, self.hidden, self.layers = n_in, hidden, layers
        self.device = torch.device(device)
        n = ctypes.c_size_t()
        check(lib.mrf_mlp_param_count(h, ctypes.byref(n)), "mrf_mlp_param_count")
        self.n_params = n.value

    def _ptrs(self):
        p, g = ctypes.c_void_p(), ctypes.c_void_p()
        check(lib.mrf_mlp_params(self.handle, ctypes.byref(p), ctypes.byref(g)), "mrf_mlp_params")
        return p.value, g.value

    def get_params(self):
        torch.cuda.synchronize()
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        check(copy_from_ptr(out, self._ptrs()[0]), "hipMemcpy")
        return out

    def get_grads(self):
        torch.cuda.synchronize()
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        check(copy_from_ptr(out, self._ptrs()[1]), "hipMemcpy")
        return out

    def set_params(self, flat):
        need(flat, torch.float32, (self.n_params,), "params")
        torch.cuda.synchronize()
        check(copy_to_ptr(self._ptrs()[0], flat), "hipMemcpy")

    def reset_optimizer(self, stream=None):
        check(lib.mrf_mlp_reset_optimizer(self.handle, stream_ptr(stream)), "mrf_mlp_reset_optimizer")

    def set_grid(self, grid, stream=None):
        """grid: mrfgen.param_grid's dict (log-spaced T1 and T2 axes, grid_index [n1, n2, nb])."""
        t1, t2 = np.log(grid["t1_axis"]), np.log(grid["t2_axis"])
        gi = torch.from_numpy(np.ascontiguousarray(grid["grid_index"][:, :, 0], np.int32)).to(self.device)
        check(lib.mrf_mlp_set_grid(self.handle, len(t1), float(t1[0]), float(t1[1] - t1[0]), len(t2), float(t2[0]),
                                   float(t2[1] - t2[0]), ptr(gi), stream_ptr(stream)), "mrf_mlp_set_grid")

    def target_stats(self, d, stream=None):
        st = (ctypes.c_double * 4)()
        check(lib.mrf_mlp_target_stats(self.handle, d.handle, st, stream_ptr(stream)), "mrf_mlp_target_stats")
        return np.array(st[:])

    def synth(self, d, seed, step, batch, snr_lo=20.0, snr_hi=60.0, stream=None):
        z = torch.empty((batch, self.n_in), dtype=torch.float32, device=self.device)
        t = torch.empty((batch, 2), dtype=torch.float32, device=self.device)
        m = torch.empty(batch, dtype=torch.int32, device=self.device)
        check(lib.mrf_mlp_synth(self.handle, d.handle, ctypes.c_uint64(seed), int(step), int(batch), float(snr_lo),
                                float(snr_hi), ptr(z), ptr(t), ptr(m), stream_ptr(stream)), "mrf_mlp_synth")
        return z, t, m

    def _ws(self, batch):
        n = ctypes.c_size_t()
        check(lib.mrf_mlp_train_workspace_size(self.handle, int(batch), ctypes.byref(n)), "mrf_mlp_train_workspace_size")
        return workspace(n.value, self.device)

    def forward(self, z, bf16=False, stream=None):
        B = z.shape[0]
        need(z, torch.float32, (B, self.n_in), "z")
        y = torch.empty((B, 2), dtype=torch.float32, device=self.device)
        ws = self._ws(B)
        check(lib.mrf_mlp_forward(self.handle, ptr(z), B, int(bf16), ptr(y), ptr(ws), ws.numel(), stream_ptr(stream)),
              "mrf_mlp_forward")
        return y

    def grads(self, z, t, bf16=False, stream=None):
        """Returns (loss, flat gradients) of one batch."""
        B = z.shape[0]
        need(z, torch.float32, (B, self.n_in), "z")
        need(t, torch.float32, (B, 2), "t")
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        ws = self._ws(B)
        check(lib.mrf_mlp_grads(self.handle, ptr(z), ptr(t), B, int(bf16), ptr(loss), ptr(ws), ws.numel(),
                                stream_ptr(stream)), "mrf_mlp_grads")
        return float(loss.item()), self.get_grads()

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        check(lib.mrf_mlp_adam_step(self.handle, float(lr), float(beta1), float(beta2), float(eps), stream_ptr(stream)),
              "mrf_mlp_adam_step")

    def train(self, d, steps, batch=4096, lr=1e-3, first_step=0, total_steps=0, cosine=True, snr_lo=20.0,
              snr_hi=60.0, seed=1, bf16=True, stream=None):
        cfg = MlpTrainCfg(int(batch), int(steps), int(first_step), int(total_steps), float(lr), 0.9, 0.999, 1e-8,
                          int(cosine), float(snr_lo), float(snr_hi), int(seed), int(bf16))
        losses = torch.empty(max(1, steps), dtype=torch.float32, device=self.device)
        ws = self._ws(batch)
        check(lib.mrf_mlp_train(self.handle, d.handle, ctypes.byref(cfg), ptr(losses), ptr(ws), ws.numel(),
                                stream_ptr(stream)), "mrf_mlp_train")
        return losses[:steps]

    def match(self, d, alpha, theta, bf16=True, stream=None):
        """Returns dict(idx, t12, rho, resid, fallback, n_fallback) for alpha [Nv, r] (complex64, device)."""
        Nv = alpha.shape[0]
        need(alpha, torch.complex64, (Nv, self.n_in // 2), "alpha")
        n = ctypes.c_size_t()
        check(lib.mrf_mlp_match_workspace_size(self.handle, Nv, ctypes.byref(n)), "mrf_mlp_match_workspace_size")
        ws = workspace(n.value, self.device)
        out = dict(idx=torch.empty(Nv, dtype=torch.int32, device=self.device),
                   t12=torch.empty((Nv, 2), dtype=torch.float32, device=self.device),
                   rho=torch.empty(Nv, dtype=torch.float32, device=self.device),
                   resid=torch.empty(Nv, dtype=torch.float32, device=self.device),
                   fallback=torch.empty(Nv, dtype=torch.int32, device=self.device))
        nfb = ctypes.c_int()
        check(lib.mrf_mlp_match(self.handle, d.handle, ptr(alpha), Nv, int(bf16), float(theta), ptr(out["idx"]),
                                ptr(out["t12"]), ptr(out["rho"]), ptr(out["resid"]), ptr(out["fallback"]),
                                ctypes.byref(nfb), ptr(ws), ws.numel(), stream_ptr(stream)), "mrf_mlp_match")
        out["n_fallback"] = nfb.value
        return out

    def save(self, stream=None):
        """The network's state (mrf_mlp_save) as a host uint8 tensor."""
        n = ctypes.c_size_t()
        check(lib.mrf_mlp_state_bytes(self.handle, ctypes.byref(n)), "mrf_mlp_state_bytes")
        buf = torch.empty(n.value, dtype=torch.uint8)
        check(lib.mrf_mlp_save(self.handle, ctypes.c_void_p(buf.data_ptr()), n.value, stream_ptr(stream)), "mrf_mlp_save")
        return buf

    def load(self, buf, stream=None):
        """Restores a state written by save (host or device uint8 tensor)."""
        check(lib.mrf_mlp_load(self.handle, ctypes.c_void_p(buf.data_ptr()), buf.numel(), stream_ptr(stream)),
              "mrf_mlp_load")

    def close(self):
        if getattr(self, "handle", None):
            lib.mrf_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
