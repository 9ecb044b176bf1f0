"""Oracle runs in worker processes (spawned: the workers never touch the GPU)."""
import multiprocessing as mp
import os

_CACHE = {}


def _qubo(key):
    import oracle
    if key not in _CACHE:
        n, F1, F2, D, penalty = key[0], key[1], key[2], key[3], key[4]
        import numpy as np
        _CACHE.clear()
        _CACHE[key] = oracle.Qubo(np.frombuffer(F1, np.int32).reshape(n, n),
                                  np.frombuffer(F2, np.int32).reshape(n, n),
                                  np.frombuffer(D, np.int32).reshape(n, n), penalty)
    return _CACHE[key]


def _job(args):
    import oracle
    key, r, kw = args
    q = _qubo(key)
    return r, oracle.run_replica(q, r, **kw)


def run_replicas(F1, F2, D, replicas, penalty=0, workers=None, **kw):
    """Oracle results for the given replica indices, computed in parallel."""
    import numpy as np
    F1 = np.ascontiguousarray(F1, np.int32)
    F2 = np.ascontiguousarray(F2, np.int32)
    D = np.ascontiguousarray(D, np.int32)
    key = (int(D.shape[0]), F1.tobytes(), F2.tobytes(), D.tobytes(), int(penalty))
    jobs = [(key, int(r), kw) for r in replicas]
    if workers is None:
        workers = min(len(jobs), max(1, min(16, (os.cpu_count() or 2) - 1)))
    if workers <= 1 or len(jobs) == 1:
        return dict(_job(j) for j in jobs)
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        return dict(pool.map(_job, jobs, chunksize=1))


_GCACHE = {}


def _gjob(args):
    import numpy as np
    import oracle
    key, r, kw = args
    if key not in _GCACHE:
        _GCACHE.clear()
        K, m, Qb, qb = key
        _GCACHE[key] = oracle.GQubo(np.frombuffer(Qb, np.int32).reshape(K, m, m), np.frombuffer(qb, np.int64))
    return r, oracle.run_greplica(_GCACHE[key], r, **kw)


def run_greplicas(Q, q, replicas, workers=None, **kw):
    """Oracle results of the K-objective MDA for the given replica indices, in parallel."""
    import numpy as np
    Q = np.ascontiguousarray(Q, np.int32)
    q = np.ascontiguousarray(q, np.int64)
    key = (int(Q.shape[0]), int(Q.shape[1]), Q.tobytes(), q.tobytes())
    jobs = [(key, int(r), kw) for r in replicas]
    if workers is None:
        workers = min(len(jobs), max(1, min(16, (os.cpu_count() or 2) - 1)))
    if workers <= 1 or len(jobs) == 1:
        return dict(_gjob(j) for j in jobs)
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        return dict(pool.map(_gjob, jobs, chunksize=1))
