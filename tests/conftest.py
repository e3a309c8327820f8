import os
import subprocess
import sys
import tempfile
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HERE = os.path.dirname(os.path.abspath(__file__))


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line(
        "markers", "slow: CPU test that takes more than ~20 s")
    config.addinivalue_line(
        "markers", "oracle_run(name): needs the long oracle run `name` of tests/oracle_runs.py, "
                   "started in the background when such a test is selected")


class OracleRuns:
    """Background processes of tests/oracle_runs.py, one per run name."""

    def __init__(self):
        self.dir = None
        self.procs = {}
        self.logs = {}

    def start(self, names):
        self.dir = tempfile.mkdtemp(prefix="lbm_oracle_runs_")
        for name in sorted(names):
            log = open(os.path.join(self.dir, name + ".log"), "w")
            self.logs[name] = log
            self.procs[name] = subprocess.Popen(
                [sys.executable, os.path.join(HERE, "oracle_runs.py"), name, self.dir],
                stdout=log, stderr=subprocess.STDOUT, cwd=ROOT)

    def wait(self, name, step, timeout=900.0):
        """The oracle's output at `step` (a dict of arrays), waiting for it."""
        import numpy as np
        if name not in self.procs:
            raise RuntimeError("oracle run %s was not started" % name)
        path = os.path.join(self.dir, "%s_%d.npz" % (name, step))
        t0 = time.time()
        while not os.path.exists(path):
            rc = self.procs[name].poll()
            if rc is not None and not os.path.exists(path):
                self.logs[name].flush()
                tail = open(os.path.join(self.dir, name + ".log")).read()[-2000:]
                raise RuntimeError("oracle run %s ended (rc %s) without step %d:\n%s"
                                   % (name, rc, step, tail))
            if time.time() - t0 > timeout:
                raise TimeoutError("oracle run %s did not reach step %d in %.0f s"
                                   % (name, step, timeout))
            time.sleep(0.5)
        with np.load(path) as z:
            return {k: z[k] for k in z.files}

    def stop(self):
        for p in self.procs.values():
            if p.poll() is None:
                p.terminate()
                try:
                    p.wait(10)
                except subprocess.TimeoutExpired:
                    p.kill()
        for f in self.logs.values():
            f.close()


_RUNS = OracleRuns()


@pytest.hookimpl(trylast=True)
def pytest_collection_modifyitems(session, config, items):
    """After deselection: start the long oracle runs the selected tests need."""
    names = set()
    for item in items:
        for m in item.iter_markers("oracle_run"):
            names.add(m.args[0])
    if names and not config.getoption("collectonly"):
        _RUNS.start(names)


def pytest_sessionfinish(session, exitstatus):
    _RUNS.stop()


@pytest.fixture(scope="session")
def oracle_runs():
    return _RUNS
