"""FP16 storage of the pyramid levels (filters and blend accumulate in FP32) against the
FP64 oracle on the whole C1 canvas, next to the FP32-storage path.

The FP16 bounds are worst-case bounds of the storage roundings, u = 2^-11 being FP16's
unit roundoff and every stored value lying in [-1, 1]:
  G_k (k >= 1) is REDUCE of the stored G_{k-1}, then stored:      e(G_k)  <= k u
  L_0 comes from G_0 and G_1 before any storage:                 e(L_0)  <= u
  L_k = G_k - EXPAND(REDUCE(G_k)) (gain <= 2), then stored:       e(L_k)  <= (2k + 1) u
  the top band is G_{L-1} itself:                                 e(L_top) <= (L - 1) u
  B_k = sum_i Gm_i L_i with sum_i Gm_i = 1, at most two cameras
  overlapping and e(Gm_k) <= k u:                                 e(B_k)  <= (2k + 1) u + 2 k u
  R_k = B_k + EXPAND(R_{k+1}) (gain 1), then stored:               e(R_k)  <= sum_{j>=k} (e(B_j) + u)
and the uint8 output moves by at most 255 e(R_0) + 1.
"""
import numpy as np
import pytest

import workloads as wl
from helpers import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]
U16 = 2.0 ** -11


def _bounds(L):
    eB = [(2 * k + 1) * U16 + 2 * k * U16 for k in range(L)]
    eB[L - 1] = (L - 1) * U16 + 2 * (L - 1) * U16
    eR = [sum(eB[j] + U16 for j in range(k, L)) for k in range(L)]
    eL = [U16] + [(2 * k + 1) * U16 for k in range(1, L - 1)] + [(L - 1) * U16]
    return eL, eR


def test_fp16_storage_error_is_within_its_rounding_bounds():
    import bench

    rig = wl.rig_c1()
    rep = bench.precision_report(rig, full=True)
    print({s: [(lv["k"], f"{lv['R_max']:.2e}", f"{lv['L_max']:.2e}") for lv in rep[s]["levels"]] for s in
           ("f32", "f16")}, rep["f16"]["u8_vs_oracle_hist"], rep["f16_vs_f32_u8_hist_full_canvas"])
    # FP32 storage: the path's own tolerance
    for lv in rep["f32"]["levels"]:
        assert lv["R_max"] <= 1e-4 and lv["L_max"] <= 1e-4, lv
    h32 = rep["f32"]["u8_vs_oracle_hist"]
    assert max(h32) <= 1 and rep["f32"]["u8_vs_oracle_frac_off"] <= 1e-4
    # FP16 storage: the rounding bounds above
    eL, eR = _bounds(rig.levels)
    for lv in rep["f16"]["levels"]:
        k = lv["k"]
        assert lv["L_max"] <= eL[k] + 1e-6, (k, lv["L_max"], eL[k])
        assert lv["R_max"] <= eR[k] + 1e-6, (k, lv["R_max"], eR[k])
    h16 = rep["f16"]["u8_vs_oracle_hist"]
    assert max(h16) <= int(np.floor(255 * eR[0] + 1))
    # and the FP16 path is not the FP32 path (its levels really are stored in FP16)
    assert any(lv["R_max"] > 1e-4 for lv in rep["f16"]["levels"])
