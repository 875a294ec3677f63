"""The C-ABI library loads and exports every entry point that
include/symrom.h declares (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "symrom.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


def _lib_path():
    from paper_2201_05555_amd import binding, _build
    if not os.path.exists(binding.LIB_PATH):
        _build.build()
    return binding.LIB_PATH


def test_header_declares_the_named_entry_points():
    names = _declared()
    for required in ("rom_init", "rom_step", "rom_adapt_rank", "fom_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2201_05555_amd import binding
    assert sorted(binding.exported_symbols()) == _declared()


def test_workspace_sizes_and_validation_on_host():
    """Size queries run on the host and reject invalid configurations."""
    from paper_2201_05555_amd import binding
    L = binding.lib()
    assert L.fom_workspace_bytes(1000, 4, 64) > 8 * 1000 * 4 * 2
    assert L.fom_workspace_bytes(0, 4, 64) == 0
    assert L.pic_workspace_bytes(10, 3, 5000) == 0          # Nx above the limit
    ok = binding.make_config(1000, 4, 64, 10)
    assert L.rom_workspace_bytes(ok) > 0
    for bad in (binding.make_config(1000, 4, 64, 9),          # odd rank
                binding.make_config(1000, 4, 64, 10, two_n_max=8),
                binding.make_config(1000, 4, 64, 70, two_n_max=70)):
        assert L.rom_workspace_bytes(bad) == 0
