"""Many independent GEMMs in one persistent launch, replayed from a HIP graph.

``GroupedPlan`` wraps mgemm_grouped_plan_* and ``tune`` the library's tuner
(mgemm_grouped_tune); argument marshalling only.  Tuned choices persist in
the library's own cache file (``tune_cache``), which it reads and writes.
"""
import ctypes
import os

from ._lib import PRECISIONS, MgemmError, Problem, check, lib
from .api import _ptr, stream_handle

NUM_BUCKETS = 4


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _problem_array(problems):
    arr = (Problem * max(1, len(problems)))()
    for i, p in enumerate(problems):
        arr[i] = Problem(p["transA"].encode(), p["transB"].encode(), p["M"], p["N"], p["K"],
                         float(p.get("alpha", 1.0)), float(p.get("beta", 0.0)),
                         _ptr(p["A"]), p["lda"], _ptr(p["B"]), p["ldb"], _ptr(p["C"]),
                         p["ldc"])
    return arr


def bucket(M, N, K=0):
    return lib().mgemm_grouped_bucket(M, N, K)


def variant_count(precision="fp32"):
    return lib().mgemm_grouped_variant_count(_prec(precision))


def variant_info(precision, v):
    b = [ctypes.c_int() for _ in range(3)]
    check(lib().mgemm_grouped_variant_info(_prec(precision), v, *[ctypes.byref(x) for x in b]))
    return dict(bm=b[0].value, bn=b[1].value, bk=b[2].value)


class GroupedPlan:
    """A plan for a list of problems.  Each problem is a dict with keys
    transA, transB, M, N, K, alpha, beta, A, lda, B, ldb, C, ldc (A, B, C:
    float32 device tensors or device addresses; the tensors must outlive
    the plan)."""

    def __init__(self, problems, precision="fp32", bucket_configs=None, tune_cache=None,
                 stream=None):
        """bucket_configs: the four bucket variants (mgemm_grouped_plan_create_ex);
        otherwise tune_cache (a path, or MGEMM_TUNE_CACHE from the
        environment) lets the library read, or tune on `stream` and store,
        them (mgemm_grouped_plan_create); neither: the library defaults."""
        self._problems = list(problems)     # keeps the tensors alive
        arr = _problem_array(self._problems)
        plan = ctypes.c_void_p()
        bad = ctypes.c_int64(-1)
        bst = ctypes.c_int(0)
        if bucket_configs is not None:
            cfg = (ctypes.c_int * NUM_BUCKETS)(*bucket_configs)
            st = lib().mgemm_grouped_plan_create_ex(arr, len(self._problems), _prec(precision),
                                                    cfg, None, ctypes.byref(plan),
                                                    ctypes.byref(bad), ctypes.byref(bst))
        else:
            cache = tune_cache if tune_cache is not None else os.environ.get("MGEMM_TUNE_CACHE")
            st = lib().mgemm_grouped_plan_create(arr, len(self._problems), _prec(precision),
                                                 cache.encode() if cache else None,
                                                 stream_handle(stream) if cache else None,
                                                 ctypes.byref(plan), ctypes.byref(bad))
        self.bad_index, self.bad_status = bad.value, bst.value
        check(st)
        self._plan = plan

    def launch(self, stream=None):
        """Replay the recorded graph on `stream` (torch's current stream by
        default)."""
        check(lib().mgemm_grouped_plan_launch(self._handle(), stream_handle(stream)))

    def run(self, stream=None):
        """Launch the persistent kernel directly (no graph)."""
        check(lib().mgemm_grouped_plan_run(self._handle(), stream_handle(stream)))

    def info(self):
        t, w = ctypes.c_int64(), ctypes.c_int64()
        check(lib().mgemm_grouped_plan_info(self._handle(), ctypes.byref(t), ctypes.byref(w)))
        return dict(tiles=t.value, workgroups=w.value)

    def close(self):
        if getattr(self, "_plan", None) is not None:
            check(lib().mgemm_grouped_plan_destroy(self._plan))
            self._plan = None

    def _handle(self):
        if self._plan is None:
            raise MgemmError(107, "plan is closed")
        return self._plan

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune(problems, precision="fp32", reps=3, stream=None):
    """Bucket configurations for this batch, measured by the library's tuner
    (which RUNS the problems and leaves every C with unspecified contents).
    Returns (configs, best milliseconds)."""
    arr = _problem_array(problems)
    cfg = (ctypes.c_int * NUM_BUCKETS)()
    ms = ctypes.c_float()
    check(lib().mgemm_grouped_tune(arr, len(problems), _prec(precision), stream_handle(stream),
                                   reps, cfg, ctypes.byref(ms)))
    return list(cfg), ms.value
