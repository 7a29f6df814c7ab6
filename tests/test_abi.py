"""CPU checks of the C ABI: the library loads, exports every declared entry point, and the
binding's record layouts match the header's structs.  No compute calls (no GPU here)."""
import ctypes
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hs_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2309_00019_amd import hs
    lib = hs.load_library()
    names = _declared()
    assert "hs_matched_filter" in names and len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(hs.EXPORTS) == names


def test_abi_version_and_error_string_without_gpu():
    from paper_2309_00019_amd import hs
    lib = hs.load_library()
    assert lib.hs_abi_version() == 10
    assert isinstance(lib.hs_last_error(), bytes)


def test_record_layouts_match_header():
    from paper_2309_00019_amd import hs
    import synth
    assert hs.CANDIDATE.itemsize == 16 and hs.TRIGGER.itemsize == 24 and hs.COINC.itemsize == 40
    assert hs.TRIGGER.fields["tick"][1] == 8 and hs.COINC.fields["tick_h"][1] == 8
    assert hs.COINC.fields["stat"][1] == 32
    assert hs.CANDIDATE == synth.CANDIDATE_DTYPE and hs.TRIGGER == synth.TRIGGER_DTYPE
    assert hs.COINC == synth.COINC_DTYPE
    assert ctypes.sizeof(hs._Bank) == 4 + 4 + 8 + 8 + 6 * 8 + 8 + 8


def test_argument_errors_need_no_gpu():
    """Null-context calls fail with HS_EINVAL before touching the device."""
    from paper_2309_00019_amd import hs
    lib = hs.load_library()
    assert lib.hs_whiten(None, None, 1024, 1.0, 0.0, None, None) == hs.HS_EINVAL
    assert lib.hs_create(None, 0, None) == hs.HS_EINVAL
    assert b"null" in lib.hs_last_error().lower()
    assert lib.hs_mlp_forward(None, None, None, 4, None) == hs.HS_EINVAL
    assert lib.hs_mlp_propose(None, None, None, 4, 0.9, 7.0, 0.5, None) == hs.HS_EINVAL
    assert lib.hs_mlp_train_step(None, None, None, None, 1, 0.01, None, None, 4, None, None) == hs.HS_EINVAL
    assert lib.hs_proposer_features(None, None, 1, None, 0, None, None, None, 0, None, None, 8, 1, None, None, 1,
                                    1, 1, 1, None) == hs.HS_EINVAL
    assert lib.hs_followup_cells(None, None, 0, 7.0, None, 0, None, None, 0, 0.05, None, None, 1, 0, None,
                                 None) == hs.HS_EINVAL
    assert lib.hs_set_mf_batch_bytes(None, 1 << 27) == hs.HS_EINVAL
    assert lib.hs_set_mf_tile(None, 128) == hs.HS_EINVAL and lib.hs_get_mf_tile(None) == 0
    assert lib.hs_set_mf_pa_cols(None, 64) == hs.HS_EINVAL and lib.hs_get_mf_pa_cols(None) == 0
    assert lib.hs_get_mf_batch_bytes(None) == 0


def test_mlp_sizes_match_header():
    from paper_2309_00019_amd import hs
    from oracle import proposer
    src = open(os.path.join(ROOT, "include", "hs.h")).read()
    vals = {k: v for k, v in re.findall(r"#define (HS_MLP_[A-Z]+) \(?([0-9]+)", src)}
    assert int(vals["HS_MLP_FEATURES"]) == hs.MLP_FEATURES == proposer.N_FEATURES
    assert int(vals["HS_MLP_CELLS"]) == hs.MLP_CELLS == proposer.N_CELLS
    assert int(vals["HS_MLP_PARAMS"]) == hs.MLP_PARAMS == proposer.N_PARAMS
    assert hs.MLP_MODEL == proposer.N_MODEL


def test_record_round_trip_helpers():
    from paper_2309_00019_amd import hs
    rec = np.zeros(3, hs.TRIGGER)
    rec["tick"] = [1, 2 ** 40, 5]
    rec["snr"] = [4.5, 5.5, 6.5]
    raw = rec.view(np.uint8).reshape(-1).view(np.int32).reshape(3, 6)
    back = raw.reshape(-1).view(np.uint8).view(hs.TRIGGER)
    assert np.array_equal(back, rec)
