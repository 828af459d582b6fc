import os
import shutil
import subprocess
import sys
import tempfile
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
    config.addinivalue_line("markers", "oracle256: needs the oracle's 256^3 reference solution (computed in a "
                                       "background process started when such a test is collected)")


class _Job:
    """The background oracle process of the full-size parity test."""

    def __init__(self):
        self.dir = tempfile.mkdtemp(prefix="oracle256_")
        self.log = open(os.path.join(self.dir, "job.log"), "w")
        self.proc = subprocess.Popen([sys.executable, os.path.join(ROOT, "tests", "oracle_ref_job.py"), self.dir],
                                     stdout=self.log, stderr=subprocess.STDOUT, cwd=ROOT)

    def wait(self, timeout_s: float):
        """Paths of the finished job's files; prints a line every 30 s while waiting."""
        t0 = time.monotonic()
        last = t0
        done = os.path.join(self.dir, "result.json")
        while not os.path.exists(done):
            if self.proc.poll() is not None and not os.path.exists(done):
                raise RuntimeError(f"oracle job ended with {self.proc.returncode}: " + self.tail())
            if time.monotonic() - t0 > timeout_s:
                raise TimeoutError("oracle job still running: " + self.tail())
            if time.monotonic() - last > 30:
                print("waiting for the oracle job:", self.tail().strip().splitlines()[-1:] or "", flush=True)
                last = time.monotonic()
            time.sleep(1.0)
        self.proc.wait()
        return self.dir

    def tail(self) -> str:
        self.log.flush()
        with open(os.path.join(self.dir, "job.log")) as f:
            return f.read()[-2000:]

    def close(self):
        if self.proc.poll() is None:
            self.proc.kill()
            self.proc.wait()
        self.log.close()
        shutil.rmtree(self.dir, ignore_errors=True)


_job = None


@pytest.hookimpl(trylast=True)
def pytest_collection_modifyitems(session, config, items):
    # after -m / -k deselection: start the reference job only if a selected test needs it
    global _job
    if _job is None and any(item.get_closest_marker("oracle256") for item in items):
        import oracle

        if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
            oracle.build(force=True)
        _job = _Job()


def pytest_unconfigure(config):
    global _job
    if _job is not None:
        _job.close()
        _job = None


@pytest.fixture(scope="session")
def oracle256():
    """Directory with rho.npy, b.npy, p.npy and result.json of the oracle's
    256^3 reference solve."""
    if _job is None:
        pytest.skip("the oracle job was not started")
    return _job.wait(timeout_s=1500)


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle

    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build(force=True)
    yield
