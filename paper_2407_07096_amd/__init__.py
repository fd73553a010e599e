"""MI355X (gfx950) Gaussian kernel density estimation, after STAG 2.0.

Exact KDE on the matrix cores, E2LSH hashing, the CKNS LSH estimator, kernel
similarity-graph edge sampling and a continuous-batching serving loop, all in
the HIP library ``libstagkde.so`` behind the C ABI of ``include/stag_kde.h``.
This package is the thin Python binding of that ABI.
"""
from ._lib import (FORMS, KERNELS, LSH_ALL_SAMPLED, LSH_LITERAL, E2LSHTable, LshIndex, Server, StagError, collision_probability,  # noqa: F401
                   declared_symbols, draws_per_node, e2lsh_hash, kde_exact, kde_lsh, kde_random_sample, kmeans, last_error, library_path, load, lsh_derive,
                   rs_sample_size, simgraph_sample, simgraph_sample_tree, spectral_cluster, spectral_embedding)

__all__ = ["FORMS", "KERNELS", "LSH_ALL_SAMPLED", "LSH_LITERAL", "E2LSHTable", "LshIndex", "Server", "StagError", "collision_probability",
           "declared_symbols", "draws_per_node", "e2lsh_hash", "kde_exact", "kde_lsh", "kde_random_sample", "kmeans", "last_error", "library_path", "load",
           "lsh_derive", "rs_sample_size", "simgraph_sample", "simgraph_sample_tree", "spectral_cluster",
           "spectral_embedding"]
