"""Static GPU index for MI355X (gfx950): sorted-array binary search (BS),
Eytzinger binary search (EBS) and Eytzinger k-ary search (EKS) with batched
point and range lookups, after Henneberg and Schuhknecht, "Bigger Is Not
Better: The Fastest Static GPU Index Is Also Lightweight!" (2025).

All work runs in the hand-written HIP kernels of ``libidx.so`` behind the C
ABI of ``include/idx.h``; this package only marshals arguments.
"""
from ._binding import (IDX_AOS, IDX_BS, IDX_EBS, IDX_EKS, IDX_ERR_ARG, IDX_ERR_CAPACITY, IDX_ERR_HIP,
                       IDX_ERR_NOMEM, IDX_ERR_RESERVED_ROWID, IDX_KEY_U32, IDX_KEY_U64, IDX_MISS, IDX_OK,
                       IDX_SOA, IDX_AOS_PADDED, LIB_PATH, SIGNATURES, IdxError, Index, idx_allocator, idx_info,
                       idx_lookup_params, lib, probe_random, IDX_FEATURE_AUTO, IDX_FEATURE_LINEAR,
                       IDX_FEATURE_LOG, IDX_FEATURE_SPLINE, idx_learn_stats, Batch, IDX_BATCH_GRAPH, learn_batch)

__all__ = [
    "Index", "IdxError", "lib", "LIB_PATH", "SIGNATURES", "idx_allocator", "idx_info", "idx_lookup_params",
    "IDX_BS", "IDX_EBS", "IDX_EKS", "IDX_KEY_U32", "IDX_KEY_U64", "IDX_SOA", "IDX_AOS", "IDX_MISS", "IDX_OK",
    "IDX_ERR_ARG", "IDX_ERR_RESERVED_ROWID", "IDX_ERR_NOMEM", "IDX_ERR_HIP", "IDX_ERR_CAPACITY",
]
