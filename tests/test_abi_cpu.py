"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and host-side validation works without a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "swcs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(swcs_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_header_symbols():
    from paper_2411_07920_amd import swcs
    lib = swcs.load()
    syms = header_symbols()
    assert len(syms) >= 25
    for name in syms:
        assert hasattr(lib, name), name
        assert name in swcs.SIGNATURES, name


def test_version_and_param_count():
    from paper_2411_07920_amd import swcs
    assert "gfx950" in swcs.version()
    assert swcs.mlp_param_count() == 16 * 128 + 128 + 128 * 128 + 128 + 128 + 1


def test_create_rejects_bad_arguments():
    from paper_2411_07920_amd import swcs
    for args in ((0, 1, 1), (33, 2, 2), (6, 7, 1), (6, 0, 0), (6, -1, 2)):
        with pytest.raises(swcs.SwcsError) as ei:
            swcs.Context(*args)
        assert ei.value.code == swcs.SWCS_E_INVALID


def test_create_without_device_is_unsupported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2411_07920_amd import swcs
    with pytest.raises(swcs.SwcsError) as ei:
        swcs.Context(6, 2, 2)
    assert ei.value.code in (swcs.SWCS_E_UNSUPPORTED, swcs.SWCS_E_DEVICE)


def test_null_context_calls_are_rejected():
    from paper_2411_07920_amd import swcs
    lib = swcs.load()
    assert lib.swcs_set_stream(None, None) == swcs.SWCS_E_INVALID
    assert lib.swcs_energy(None, None, None, None) == swcs.SWCS_E_INVALID
    lib.swcs_destroy(None)


def test_kernel_timer_ids_match_header():
    """The binding's kernel names map to the header's SWCS_K_* values."""
    from paper_2411_07920_amd import swcs
    text = open(os.path.join(ROOT, "include", "swcs.h")).read()
    ids = {m.group(1).lower(): int(m.group(2)) for m in re.finditer(r"SWCS_K_([A-Z_]+)\s*=\s*(\d+)", text)}
    assert sorted(ids.values()) == list(range(1, len(ids) + 1))
    assert sorted(swcs.KERNELS.values()) == sorted(ids.values())
    for name, kid in swcs.KERNELS.items():
        assert ids.get(name) == kid, name
