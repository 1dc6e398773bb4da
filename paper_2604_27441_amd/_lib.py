"""ctypes declarations mirroring include/revo.h, include/revo_ops.h and include/revo_train.h."""
import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librevo.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it first (python paper_2604_27441_amd/build.py "
        "or __graft_entry__.build()); there is no fallback path")

lib = C.CDLL(LIB_PATH)

REVO_OK, REVO_EAGAIN = 0, 1
REVO_DEVICE_PTRS, REVO_HOLD = 0x1, 0x2
REVO_CFG_SHED, REVO_CFG_PROFILE, REVO_CFG_ONE_STREAM, REVO_CFG_GRAPHS = 0x1, 0x2, 0x4, 0x8
REVO_CFG_PROFILE_ATTN = 0x10
REVO_DONE, REVO_SHED, REVO_FAILED = 0, 1, 2
REVO_FRAME_U8, REVO_FRAME_U16, REVO_FRAME_F32 = 0, 1, 2


class RevoConfig(C.Structure):
    _fields_ = [
        ("device", C.c_int), ("precision", C.c_int), ("k", C.c_int), ("tubelet", C.c_int),
        ("enc_depth", C.c_int), ("dec_depth", C.c_int), ("composite", C.c_int),
        ("max_streams", C.c_int), ("max_batch", C.c_int), ("max_batch_tokens", C.c_int),
        ("hbm_budget_bytes", C.c_size_t), ("fps", C.c_float),
        ("weights_rgb", C.POINTER(C.c_float)), ("n_weights_rgb", C.c_size_t),
        ("weights_depth", C.POINTER(C.c_float)), ("n_weights_depth", C.c_size_t),
        ("flags", C.c_uint), ("hip_stream", C.c_void_p),
    ]


class RevoRequest(C.Structure):
    _fields_ = [
        ("stream_id", C.c_uint), ("frame_index", C.c_longlong), ("width", C.c_int), ("height", C.c_int),
        ("flags", C.c_uint),
        ("rgb", C.c_void_p), ("mask_rgb", C.c_void_p), ("depth", C.c_void_p), ("mask_depth", C.c_void_p),
        ("rgb_out", C.c_void_p), ("depth_out", C.c_void_p),
        ("rgb_out_f32", C.c_void_p), ("depth_out_f32", C.c_void_p),
        ("deadline_ns", C.c_longlong),
    ]


class RevoCompletion(C.Structure):
    _fields_ = [
        ("ticket", C.c_ulonglong), ("stream_id", C.c_uint), ("frame_index", C.c_longlong),
        ("status", C.c_int), ("error", C.c_int), ("submit_ns", C.c_longlong), ("done_ns", C.c_longlong),
    ]


class RevoStats(C.Structure):
    _fields_ = [
        ("batches", C.c_longlong), ("served", C.c_longlong), ("shed", C.c_longlong), ("failed", C.c_longlong),
        ("attn_launches", C.c_longlong), ("attn_ms", C.c_double), ("attn_flop", C.c_double),
        ("gemm_launches", C.c_longlong), ("gemm_ms", C.c_double), ("gemm_flop", C.c_double),
        ("other_launches", C.c_longlong), ("other_ms", C.c_double), ("forward_ms", C.c_double),
        ("hbm_fixed_bytes", C.c_longlong), ("hbm_pool_bytes", C.c_longlong),
    ]


class RevoTrainConfig(C.Structure):
    _fields_ = [
        ("device", C.c_int), ("channels", C.c_int), ("k", C.c_int), ("tubelet", C.c_int),
        ("enc_depth", C.c_int), ("dec_depth", C.c_int), ("batch", C.c_int), ("height", C.c_int), ("width", C.c_int),
        ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float), ("tv_weight", C.c_float),
        ("weights", C.POINTER(C.c_float)), ("n_weights", C.c_size_t),
    ]


class RevoTrainBatch(C.Structure):
    _fields_ = [
        ("refs", C.c_void_p), ("target", C.c_void_p), ("mask", C.c_void_p),
        ("ref_idx", C.POINTER(C.c_longlong)), ("t_target", C.POINTER(C.c_longlong)),
    ]


_sigs = {
    "revo_config_default": (None, [C.POINTER(RevoConfig)]),
    "revo_weight_count": (C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int]),
    "revo_recover_create": (C.c_int, [C.POINTER(RevoConfig), C.POINTER(C.c_void_p)]),
    "revo_recover_submit": (C.c_int, [C.c_void_p, C.POINTER(RevoRequest), C.POINTER(C.c_ulonglong)]),
    "revo_recover_poll": (C.c_int, [C.c_void_p, C.POINTER(RevoCompletion), C.c_int, C.c_int]),
    "revo_recover_destroy": (None, [C.c_void_p]),
    "revo_strerror": (C.c_char_p, [C.c_int]),
    "revo_get_stats": (C.c_int, [C.c_void_p, C.POINTER(RevoStats), C.c_int]),
    "revo_calibrate": (C.c_int, [C.c_void_p, C.c_int]),
    "revo_op_linear": (C.c_int, [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_int, C.c_int, C.c_int, C.c_void_p]),
    "revo_op_linear_fp8": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p]),
    "revo_op_layernorm": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                    C.c_void_p]),
    "revo_op_attention": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                    C.c_int, C.c_void_p]),
    "revo_op_attention_fp8": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                        C.c_void_p, C.c_void_p]),
    "revo_op_attention_noalloc": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                            C.c_int, C.c_int, C.c_void_p]),
    "revo_train_create": (C.c_int, [C.POINTER(RevoTrainConfig), C.POINTER(C.c_void_p)]),
    "revo_train_step": (C.c_int, [C.c_void_p, C.POINTER(RevoTrainBatch), C.POINTER(C.c_double)]),
    "revo_train_get_weights": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "revo_train_get_grads": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "revo_train_get_pred": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "revo_train_destroy": (None, [C.c_void_p]),
    "revo_op_convert": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_longlong, C.c_void_p]),
    "revo_op_frame_metrics": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                        C.c_void_p, C.c_void_p]),
    "revo_op_unproject": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "revo_op_render_view": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                      C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sigs)


class RevoError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {lib.revo_strerror(code).decode()} ({code})")


def check(rc, what="revo"):
    if rc < 0:
        raise RevoError(rc, what)
    return rc
