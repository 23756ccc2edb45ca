"""C-ABI checks that need no GPU: the library loads, exports every function the
header declares, and rejects invalid arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1503_00330_amd as pi
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pi2rh.h")


def _gpu_visible():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names) - {"if", "while", "for", "return", "sizeof"})


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lwpr_predict", "pi_rollout_cost", "pi_update", "pi_rollout_adjoint",
                 "pi_rh_shift", "pi_rollout_cost_batched", "pi_workspace_bytes", "pi_last_error"):
        assert must in names
    assert sorted(pi.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(pi.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert "gfx950" in pi.version()


# Fake, never-dereferenced device addresses: every call below must fail in
# validation, before any device work.
FAKE = 0x10000


def _structs(dtype=np.float32, dyn=synth.DYN_QUAD12):
    prob, model = synth.tiny_problem(0, dyn=dyn, L=3, K=4, T=3, dtype=dtype)
    ps = pi.pi_problem()
    ps.dtype = pi.PI_F32 if dtype == np.float32 else pi.PI_F64
    ps.dyn, ps.K, ps.T, ps.M = prob.dyn, prob.K, prob.T, prob.M
    ps.dt, ps.lambda_ = prob.dt, prob.lam
    for a in range(prob.n_u):
        ps.noise_std[a] = prob.noise_std[a]
    ps.obs_kind, ps.n_obs, ps.obs = 0, prob.n_obs, FAKE
    ps.obs_penalty, ps.obs_decay = 1000.0, 10.0
    ps.seed = 1
    ms = pi.pi_lwpr()
    ms.dtype = ps.dtype
    ms.d, ms.n_out, ms.R = model.d, model.n_out, model.R
    for i in range(pi.PI_MAX_OUT + 1):
        ms.L_off[i] = int(model.L_off[min(i, model.n_out)])
    ms.centre = ms.metric = ms.proj_u = ms.beta = ms.sigma2 = FAKE
    ms.proj_p = None
    return ps, ms


def _rollout(ps, ms, ws=FAKE, ws_bytes=1 << 30, cost=FAKE):
    lib = pi.load()
    return lib.pi_rollout_cost(C.byref(ps), C.byref(ms), FAKE, FAKE, FAKE, cost, ws, ws_bytes, None)


@pytest.mark.skipif(_gpu_visible(), reason="validation-only test; runs where no GPU is visible")
class TestValidation:
    def test_null_pointers(self):
        ps, ms = _structs()
        assert _rollout(ps, ms, cost=None) == 1
        assert "non-NULL" in pi.last_error()
        lib = pi.load()
        assert lib.pi_rollout_cost(None, C.byref(ms), FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 30, None) == 1
        ms.centre = None
        assert _rollout(ps, ms) == 1

    @pytest.mark.parametrize("field,value,code", [
        ("K", 0, 2), ("T", 0, 2), ("M", -1, 2), ("dt", 0.0, 3), ("lambda_", -1.0, 3),
        ("dyn", 7, 3), ("obs_kind", 5, 3), ("n_obs", 65, 2), ("weighting", 3, 3),
        ("variant", 9, 3), ("tile_samples", 100, 3), ("tile_waves", 5, 3), ("tile_split", 3, 3),
        ("tile_split", -1, 3), ("dtype", 5, 4)])
    def test_bad_problem_fields(self, field, value, code):
        ps, ms = _structs()
        setattr(ps, field, value)
        assert _rollout(ps, ms) == code, pi.last_error()

    def test_describe_validates(self):
        ps, ms = _structs()
        lib = pi.load()
        out = (C.c_int32 * 4)()
        assert lib.pi_rollout_describe(C.byref(ps), C.byref(ms), None) == 1
        assert lib.pi_rollout_describe(None, C.byref(ms), out) == 1
        ps.tile_split = 7
        assert lib.pi_rollout_describe(C.byref(ps), C.byref(ms), out) == 3

    def test_model_fold_validates(self):
        ps, ms = _structs()
        lib = pi.load()
        n = lib.pi_model_fold_bytes(C.byref(ms))
        assert 0 < n < (1 << 40)
        assert lib.pi_model_fold(C.byref(ms), None, n, None) == 1
        assert lib.pi_model_fold(C.byref(ms), FAKE, n - 1, None) == 5
        ms.folded, ms.folded_bytes = FAKE, n - 1      # too small a folded buffer
        assert _rollout(ps, ms) == 5
        ms.d = 0
        assert lib.pi_model_fold_bytes(C.byref(ms)) == C.c_size_t(-1).value

    def test_models_past_2gib_of_tiles_keep_the_direct_form(self):
        # d = 16: one tile of 16 models takes 11 KB of matrix-core fragments, a
        # model 680 B in the direct form; tile offsets are 32-bit
        ps, ms = _structs()
        lib = pi.load()
        assert ms.d == 16

        def fold_bytes(L):      # L models spread over the quadrotor's 6 outputs
            for o in range(7):
                ms.L_off[o] = o * (L // 6)
            return lib.pi_model_fold_bytes(C.byref(ms))
        assert ms.n_out == 6
        assert fold_bytes(1 << 20) > 1.4e9          # 713 MB direct + 738 MB of tiles
        assert fold_bytes(1 << 22) < 3.0e9          # 2.85 GB direct only (tiles would be 2.95 GB)
        ps.variant = pi.PI_VARIANT_MFMA
        assert _rollout(ps, ms) == 7 and "2 GiB" in pi.last_error()

    def test_bad_model(self):
        ps, ms = _structs()
        ms.d = 17
        assert _rollout(ps, ms) == 2
        ps, ms = _structs()
        ms.L_off[2] = ms.L_off[1]           # an output with no models
        assert _rollout(ps, ms) == 2
        ps, ms = _structs()
        ms.n_out = 5                          # quadrotor needs 6 accelerations
        assert _rollout(ps, ms) == 2
        ps, ms = _structs()
        ms.dtype = pi.PI_F64                  # problem is float32
        assert _rollout(ps, ms) == 4

    def test_negative_noise(self):
        ps, ms = _structs()
        ps.noise_std[1] = -0.1
        assert _rollout(ps, ms) == 3

    def test_control_terms_need_the_hybrid_rate_channel(self):
        # the control terms of S-tilde need a control-affine channel (the hybrid
        # model's commanded rates) and R = lambda diag(1/sigma^2)/dt finite
        ps, ms = _structs()
        ps.ctrl_cost = 1
        assert _rollout(ps, ms) == 7 and "hybrid" in pi.last_error()
        ps, ms = _structs(dyn=synth.DYN_QUAD_HYBRID)
        ps.ctrl_cost = 2
        assert _rollout(ps, ms) == 3
        ps.ctrl_cost = 1
        ps.noise_std[1] = 0.0
        assert _rollout(ps, ms) == 3 and "noise_std[1]" in pi.last_error()
        ps.noise_std[1] = 0.3
        assert _rollout(ps, ms) == 6          # valid: reaches the device check

    def test_workspace_too_small(self):
        ps, ms = _structs()
        need = pi.load().pi_workspace_bytes(pi.PI_OP_ROLLOUT, C.byref(ps), C.byref(ms))
        assert 0 < need < (1 << 40)
        assert _rollout(ps, ms, ws_bytes=need - 1) == 5
        assert _rollout(ps, ms, ws=None) == 5

    def test_noalloc_rollout_validates_before_the_device(self):
        # the allocation-free rollout takes no workspace: it checks its request
        # against the static scratch and never reaches the device when too big
        lib = pi.load()
        ps, ms = _structs()
        call = lambda cost=FAKE: lib.pi_rollout_cost_noalloc(C.byref(ps), C.byref(ms), FAKE, FAKE,
                                                             FAKE, cost, None)
        assert call(cost=None) == 1
        ps.K, ps.T, ps.M = 4096, 200, 8          # 26 MB of sub-rollout costs: fits
        ps.tile_split = 1                        # (no pair-exchange slots)
        assert lib.pi_workspace_bytes(pi.PI_OP_ROLLOUT, C.byref(ps), C.byref(ms)) <= 32 << 20
        assert call() == 6 and "device" in pi.last_error()
        ps.M = 16                                # 52 MB: over the 32 MiB scratch
        assert lib.pi_workspace_bytes(pi.PI_OP_ROLLOUT, C.byref(ps), C.byref(ms)) > 32 << 20
        assert call() == 5 and "allocation-free" in pi.last_error()
        ps.K = 0
        assert call() == 2

    def test_batched_validation_names_the_problem(self):
        # the batch's messages carry the problem index once, ahead of the
        # problem's own message (copied, not formatted into itself)
        lib = pi.load()
        ps0, ms0 = _structs()
        ps1, ms1 = _structs()
        ps1.tile_samples = 128                     # float32 products: 32 at most
        PS, MS = pi.pi_problem * 2, pi.pi_lwpr * 2
        n = lib.pi_batched_workspace_bytes(2, PS(ps0, ps1), MS(ms0, ms1))
        assert n == C.c_size_t(-1).value
        assert pi.last_error() == "problem 1: tile_samples=128 outside [0,32]"
        ps1.tile_samples, ps1.variant = 128, pi.PI_VARIANT_MFMA_BF16X3   # bf16 form: 128 allowed
        ps0.variant = pi.PI_VARIANT_MFMA_BF16X3
        assert lib.pi_batched_workspace_bytes(2, PS(ps0, ps1), MS(ms0, ms1)) != C.c_size_t(-1).value

    def test_bf16x3_tile_limits(self):
        ps, ms = _structs()
        ps.variant, ps.tile_samples = pi.PI_VARIANT_MFMA_BF16X3, 129
        assert _rollout(ps, ms) == 3 and "outside [0,128]" in pi.last_error()
        ps.tile_samples, ps.tile_waves = 32, 8        # 8 waves: <= 16 or the 128-row shared tile
        assert _rollout(ps, ms) == 7
        ps.tile_samples = 128
        assert _rollout(ps, ms) == 6 and "device" in pi.last_error()   # valid: only the device is missing

    def test_adjoint_pieces_forward_needs_the_quadrotor(self):
        # the adjoint runs its forward in the requested pieces form only for
        # the float32 12-state quadrotor with d = 16
        lib = pi.load()

        def adjoint(ps, ms):
            return lib.pi_rollout_adjoint(C.byref(ps), C.byref(ms), FAKE, FAKE, FAKE, 0, None, FAKE, FAKE, FAKE,
                                          FAKE, FAKE, 1 << 30, None)
        for v in (pi.PI_VARIANT_MFMA_F16X2, pi.PI_VARIANT_MFMA_BF16X3):
            ps, ms = _structs(dyn=synth.DYN_POINTMASS2D)
            ps.variant = v
            assert adjoint(ps, ms) == 7 and "forward needs the float32 12-state quadrotor" in pi.last_error()
            ps, ms = _structs()
            ps.variant = v
            assert adjoint(ps, ms) == 6 and "device" in pi.last_error()   # valid: only the device is missing

    def test_f16x2_tile_limits(self):
        # the two-piece fp16 form: the bf16 form's launch shapes
        for fields, code in ((dict(tile_samples=32, tile_waves=8), 7), (dict(tile_samples=129), 3),
                             (dict(tile_samples=32), 6), (dict(tile_samples=16, tile_waves=8), 6),
                             (dict(tile_split=2), 6), (dict(tile_samples=64, tile_waves=4), 6), (dict(), 6)):
            ps, ms = _structs()
            ps.variant = pi.PI_VARIANT_MFMA_F16X2
            for k, v in fields.items():
                setattr(ps, k, v)
            assert _rollout(ps, ms) == code, (fields, pi.last_error())
            if code == 7:
                assert "f16x2" in pi.last_error()

    def test_mfma_needs_float32(self):
        ps, ms = _structs(dtype=np.float64)
        ps.variant = pi.PI_VARIANT_MFMA
        assert _rollout(ps, ms) == 7

    def test_valid_call_reports_missing_device(self):
        ps, ms = _structs()
        assert _rollout(ps, ms) == 6
        assert "device" in pi.last_error()

    def test_update_and_predict_validation(self):
        lib = pi.load()
        ps, ms = _structs()
        assert lib.pi_update(C.byref(ps), None, FAKE, FAKE, None, FAKE, 1 << 30, None) == 1
        assert lib.lwpr_predict(C.byref(ms), FAKE, -1, FAKE, FAKE, 0, FAKE, 1 << 30, None) == 2
        assert lib.lwpr_predict(C.byref(ms), FAKE, 5, FAKE, FAKE, 5, FAKE, 1 << 30, None) == 3
        for v in (pi.PI_VARIANT_MFMA_BF16X3, pi.PI_VARIANT_MFMA_F16X2):   # rollouts only
            assert lib.lwpr_predict(C.byref(ms), FAKE, 5, FAKE, FAKE, v, FAKE, 1 << 30, None) == 7
        ms.d = 5
        assert lib.lwpr_predict(C.byref(ms), FAKE, 5, FAKE, FAKE, pi.PI_VARIANT_MFMA, FAKE,
                                1 << 30, None) == 7
        assert lib.pi_workspace_bytes(99, C.byref(ps), C.byref(ms)) == C.c_size_t(-1).value


def test_workspace_sizes_scale_with_problem():
    ps, ms = _structs()
    lib = pi.load()
    a = lib.pi_workspace_bytes(pi.PI_OP_UPDATE, C.byref(ps), None)
    ps.K *= 10
    assert lib.pi_workspace_bytes(pi.PI_OP_UPDATE, C.byref(ps), None) > a
    ps.M = 3     # sub-rollouts need room for per-sub-rollout costs
    r3 = lib.pi_workspace_bytes(pi.PI_OP_ROLLOUT, C.byref(ps), C.byref(ms))
    ps.M = 1
    assert r3 > lib.pi_workspace_bytes(pi.PI_OP_ROLLOUT, C.byref(ps), C.byref(ms))
    # pair-capable float32 plans reserve the exchange slots whatever the device
    ps.dtype, ms.dtype = pi.PI_F32, pi.PI_F32
    paired = lib.pi_workspace_bytes(pi.PI_OP_ROLLOUT, C.byref(ps), C.byref(ms))
    ps.tile_split = 1
    single = lib.pi_workspace_bytes(pi.PI_OP_ROLLOUT, C.byref(ps), C.byref(ms))
    assert paired > single > 0
