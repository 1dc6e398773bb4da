"""Python face of the C ABI: a Recoverer holds one revo_ctx, a Trainer one revo_trainer."""
import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import lib, check, RevoConfig, RevoRequest, RevoCompletion, RevoTrainConfig, RevoTrainBatch

REVO_FP32, REVO_BF16, REVO_FP8 = 0, 1, 2


@dataclass
class Completion:
    ticket: int
    stream_id: int
    frame_index: int
    status: int
    error: int
    submit_ns: int
    done_ns: int


def _ptr(x):
    """Address of a numpy array or a torch tensor (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous")
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return x.data_ptr()
    raise TypeError(type(x))


class Recoverer:
    """revo_recover_create / submit / poll / destroy."""

    def __init__(self, weights_rgb, weights_depth, precision=REVO_BF16, device=0, k=5, tubelet=2,
                 enc_depth=0, dec_depth=0, composite=1, max_streams=64, max_batch=16, max_batch_tokens=0,
                 hbm_budget_bytes=0, fps=30.0, shed=False, profile=False, one_stream=False,
                 graphs=False, hip_stream=None):
        cfg = RevoConfig()
        lib.revo_config_default(C.byref(cfg))
        self._w = [np.ascontiguousarray(weights_rgb, np.float32), np.ascontiguousarray(weights_depth, np.float32)]
        cfg.device, cfg.precision, cfg.k, cfg.tubelet = device, precision, k, tubelet
        cfg.enc_depth, cfg.dec_depth, cfg.composite = enc_depth, dec_depth, composite
        cfg.max_streams, cfg.max_batch, cfg.max_batch_tokens = max_streams, max_batch, max_batch_tokens
        cfg.hbm_budget_bytes, cfg.fps = hbm_budget_bytes, fps
        # profile: False, True (every kernel) or "attention" (attention launches
        # and whole passes only, which barely perturbs throughput)
        prof_flag = _lib.REVO_CFG_PROFILE_ATTN if profile == "attention" else (_lib.REVO_CFG_PROFILE if profile else 0)
        cfg.flags = ((_lib.REVO_CFG_SHED if shed else 0) | prof_flag
                     | (_lib.REVO_CFG_ONE_STREAM if one_stream else 0) | (_lib.REVO_CFG_GRAPHS if graphs else 0))
        cfg.hip_stream = hip_stream
        cfg.weights_rgb = self._w[0].ctypes.data_as(C.POINTER(C.c_float))
        cfg.n_weights_rgb = self._w[0].size
        cfg.weights_depth = self._w[1].ctypes.data_as(C.POINTER(C.c_float))
        cfg.n_weights_depth = self._w[1].size
        h = C.c_void_p()
        check(lib.revo_recover_create(C.byref(cfg), C.byref(h)), "revo_recover_create")
        self._h = h
        self._keep = {}

    def submit(self, stream_id, frame_index, width, height, rgb=None, mask_rgb=None, depth=None, mask_depth=None,
               rgb_out=None, depth_out=None, rgb_out_f32=None, depth_out_f32=None, device_ptrs=False,
               hold=False, deadline_ns=0):
        """Queue one frame; returns the ticket, or None when the queue is full."""
        r = RevoRequest()
        r.stream_id, r.frame_index, r.width, r.height = stream_id, frame_index, width, height
        r.flags = (_lib.REVO_DEVICE_PTRS if device_ptrs else 0) | (_lib.REVO_HOLD if hold else 0)
        r.rgb, r.mask_rgb, r.depth, r.mask_depth = _ptr(rgb), _ptr(mask_rgb), _ptr(depth), _ptr(mask_depth)
        r.rgb_out, r.depth_out = _ptr(rgb_out), _ptr(depth_out)
        r.rgb_out_f32, r.depth_out_f32 = _ptr(rgb_out_f32), _ptr(depth_out_f32)
        r.deadline_ns = deadline_ns
        t = C.c_ulonglong()
        rc = lib.revo_recover_submit(self._h, C.byref(r), C.byref(t))
        if rc == _lib.REVO_EAGAIN:
            return None
        check(rc, "revo_recover_submit")
        # outputs must outlive the call until poll reports the ticket
        self._keep[t.value] = (rgb_out, depth_out, rgb_out_f32, depth_out_f32)
        return t.value

    def poll(self, max_n=64, timeout_us=-1):
        buf = (RevoCompletion * max_n)()
        n = check(lib.revo_recover_poll(self._h, buf, max_n, timeout_us), "revo_recover_poll")
        out = []
        for i in range(n):
            c = buf[i]
            self._keep.pop(c.ticket, None)
            out.append(Completion(c.ticket, c.stream_id, c.frame_index, c.status, c.error, c.submit_ns, c.done_ns))
        return out

    def wait(self, tickets, timeout_us=120_000_000):
        """Poll until every ticket in `tickets` has completed; returns {ticket: Completion}."""
        want = set(tickets)
        got = {}
        while want:
            cs = self.poll(64, timeout_us)
            if not cs:
                raise TimeoutError(f"tickets {sorted(want)} did not complete")
            for c in cs:
                got[c.ticket] = c
                want.discard(c.ticket)
        return got

    def calibrate(self, phase):
        """FP8 calibration: phase 1 starts recording activation maxima, phase 0
        turns them into scales and switches the FP8 form on (revo_calibrate)."""
        check(lib.revo_calibrate(self._h, int(phase)), "revo_calibrate")

    def stats(self, reset=False):
        """Counters of the context (revo_get_stats) as a dict."""
        st = _lib.RevoStats()
        check(lib.revo_get_stats(self._h, C.byref(st), 1 if reset else 0), "revo_get_stats")
        return {name: getattr(st, name) for name, _ in st._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib.revo_recover_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def weight_count(channels, tubelet=2, enc_depth=12, dec_depth=4):
    return int(lib.revo_weight_count(channels, tubelet, enc_depth, dec_depth))


class Trainer:
    """revo_train_create / step / get_* / destroy: the FP32 pretraining step
    of one modality's model (channels 3 RGB, 1 depth) at a fixed batch shape."""

    def __init__(self, weights, channels, batch, height, width, device=0, k=5, tubelet=2, enc_depth=12,
                 dec_depth=4, lr=0.0, beta1=0.0, beta2=0.0, eps=0.0, tv_weight=0.0):
        self._w = np.ascontiguousarray(weights, dtype=np.float32)
        cfg = RevoTrainConfig(device=device, channels=channels, k=k, tubelet=tubelet, enc_depth=enc_depth,
                              dec_depth=dec_depth, batch=batch, height=height, width=width, lr=lr, beta1=beta1,
                              beta2=beta2, eps=eps, tv_weight=tv_weight,
                              weights=self._w.ctypes.data_as(C.POINTER(C.c_float)), n_weights=self._w.size)
        h = C.c_void_p()
        check(lib.revo_train_create(C.byref(cfg), C.byref(h)), "revo_train_create")
        self._h = h
        self.count = self._w.size
        self.pred_count = batch * height * width * channels
        self.shape = (batch, height, width, channels)

    def step(self, refs, target, mask, ref_idx, t_target):
        """refs / target / mask: contiguous device tensors (see revo_train.h);
        ref_idx [batch][k], t_target [batch]: host integers.  Returns the loss."""
        ri = np.ascontiguousarray(ref_idx, dtype=np.int64)
        tt = np.ascontiguousarray(t_target, dtype=np.int64)
        b = RevoTrainBatch(refs=_ptr(refs), target=_ptr(target), mask=_ptr(mask),
                           ref_idx=ri.ctypes.data_as(C.POINTER(C.c_longlong)),
                           t_target=tt.ctypes.data_as(C.POINTER(C.c_longlong)))
        loss = C.c_double()
        check(lib.revo_train_step(self._h, C.byref(b), C.byref(loss)), "revo_train_step")
        return loss.value

    def _get(self, fn, n):
        out = np.empty(n, np.float32)
        check(fn(self._h, out.ctypes.data, n), fn.__name__)
        return out

    def weights(self):
        return self._get(lib.revo_train_get_weights, self.count)

    def grads(self):
        return self._get(lib.revo_train_get_grads, self.count)

    def pred(self):
        return self._get(lib.revo_train_get_pred, self.pred_count).reshape(self.shape)

    def close(self):
        if getattr(self, "_h", None):
            lib.revo_train_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
