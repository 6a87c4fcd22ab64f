import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

LIB = os.path.join(ROOT, "paper_2205_11226_amd", "libskmmse.so")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def pytest_sessionstart(session):
    # tests use what is built; only build when nothing is there (CPU container)
    if not os.path.exists(LIB):
        import importlib.util
        path = os.path.join(ROOT, "paper_2205_11226_amd", "build.py")
        spec = importlib.util.spec_from_file_location("_skm_build", path)
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
