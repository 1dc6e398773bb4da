"""The C-ABI library loads and exports every function include/*.h declares
(no GPU work: nothing here touches a device)."""
import ctypes
import glob
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for m in re.finditer(r"\b(revo_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_function():
    import paper_2604_27441_amd as pkg
    names = _declared()
    assert {"revo_recover_create", "revo_recover_submit", "revo_recover_poll", "revo_recover_destroy"} <= names
    for n in names:
        assert hasattr(pkg.lib, n), n
    assert set(pkg._lib.EXPORTED) == names


def test_strerror_and_weight_count():
    import paper_2604_27441_amd as pkg
    import synth
    assert pkg.lib.revo_strerror(-61).decode().startswith("no clean reference")
    assert pkg.lib.revo_strerror(12345).decode() == "unknown error"
    for C in (3, 1):
        for T, ne, nd in [(2, 12, 4), (2, 2, 1), (1, 3, 2), (3, 0, 0)]:
            assert pkg.api.weight_count(C, T, ne, nd) == synth.weight_count(C, tubelet=T, enc_depth=ne, dec_depth=nd)
    assert pkg.lib.revo_weight_count(2, 2, 12, 4) == 0


def test_config_struct_matches_header_defaults():
    import paper_2604_27441_amd as pkg
    cfg = pkg._lib.RevoConfig()
    pkg.lib.revo_config_default(ctypes.byref(cfg))
    assert (cfg.precision, cfg.k, cfg.tubelet, cfg.composite) == (1, 5, 2, 1)
    assert abs(cfg.fps - 30.0) < 1e-6
    # the ctypes mirror has the C layout: weights pointer after fps (with padding)
    assert pkg._lib.RevoConfig.weights_rgb.offset == 56


def test_null_arguments_are_rejected_without_a_device():
    import paper_2604_27441_amd as pkg
    assert pkg.lib.revo_recover_create(None, None) == -22
    assert pkg.lib.revo_recover_submit(None, None, None) == -22
    assert pkg.lib.revo_recover_poll(None, None, 0, 0) == -22
    assert pkg.lib.revo_op_linear(7, 0, None, None, None, None, 1, 64, 64, None) == -95
    assert pkg.lib.revo_op_attention(1, None, None, None, None, 1, 1, 65, None) == -22


def test_trainer_null_arguments_are_rejected_without_a_device():
    import ctypes as C
    import paper_2604_27441_amd as pkg
    assert pkg.lib.revo_train_create(None, None) == -22
    assert pkg.lib.revo_train_step(None, None, None) == -22
    assert pkg.lib.revo_train_get_weights(None, None, 0) == -22
    cfg = pkg._lib.RevoTrainConfig(channels=2, k=5, tubelet=2, batch=1, height=16, width=16)
    h = C.c_void_p()
    assert pkg.lib.revo_train_create(C.byref(cfg), C.byref(h)) == -22 and not h.value
