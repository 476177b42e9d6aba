"""Parallel generation of many seeded problems (process pool, before any GPU use)."""
import os
from concurrent.futures import ProcessPoolExecutor

from .problems import star_problem


def _star(args):
    n_tri, seed, kinds = args
    return star_problem(n_tri, seed, kinds=kinds)


def stars(specs, workers=None):
    """specs: list of (n_triangles, seed, kinds). Returns the problems in order."""
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if workers <= 1 or len(specs) <= 1:
        return [_star(s) for s in specs]
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        return list(ex.map(_star, specs, chunksize=1))
