"""CPU test of the benchmark's command line: a request for several GPUs is
refused with a message and status 2 before anything touches a device."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_cli", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_several_gpus_refused(capsys):
    assert _bench().main(["--gpus", "2"]) == 2
    assert "one GPU only" in capsys.readouterr().err
