// Slot accessors for the two physical layouts (Section 7.1):
//   SoA: keys[s] and rowids[s] in two arrays;
//   AoS: blocks of `node` slots, each block holding its node keys followed by
//        its node rowids (node = k - 1 for EKS, 1 for BS/EBS), so a node's
//        keys stay contiguous and the footprint equals SoA; optionally each
//        block is padded to a power of two bytes (`stride`) so it occupies
//        whole cache lines.
// 64-bit keys in AoS blocks may be only 4-byte aligned; they are moved as two
// 32-bit words.
#pragma once

#include "internal.hpp"

namespace idx {

template <typename K, bool AOS>
struct Load;

template <typename K>
struct Load<K, false> {
    const K *__restrict__ k;
    const uint32_t *__restrict__ r;
    uint32_t node;
    __device__ __forceinline__ K key(uint64_t s) const { return k[s]; }
    __device__ __forceinline__ uint32_t row(uint64_t s) const { return r[s]; }
    // slot j of node c (slot c*node + j)
    __device__ __forceinline__ K nkey(uint64_t c, uint32_t j) const { return k[c * node + j]; }
    __device__ __forceinline__ uint32_t nrow(uint64_t c, uint32_t j) const { return r[c * node + j]; }
    __device__ __forceinline__ const K *node_ptr(uint64_t c) const { return k + c * node; }
};

template <typename K>
__device__ __forceinline__ K load_key_words(const char *p) {
    if constexpr (sizeof(K) == 8) {
        const uint32_t *w = (const uint32_t *)p;
        return ((uint64_t)w[1] << 32) | w[0];
    } else {
        return *(const uint32_t *)p;
    }
}

template <typename K>
__device__ __forceinline__ void store_key_words(char *p, K v) {
    if constexpr (sizeof(K) == 8) {
        uint32_t *w = (uint32_t *)p;
        w[0] = (uint32_t)v;
        w[1] = (uint32_t)(v >> 32);
    } else {
        *(uint32_t *)p = v;
    }
}

template <typename K>
struct Load<K, true> {
    const char *__restrict__ base;
    const uint32_t *r_unused;
    uint32_t node;
    uint32_t stride;  // bytes per block: node * (sizeof(K) + 4), or padded to a power of two
    __device__ __forceinline__ uint64_t block_bytes() const { return stride; }
    __device__ __forceinline__ K nkey(uint64_t c, uint32_t j) const {
        return load_key_words<K>(base + c * block_bytes() + (uint64_t)j * sizeof(K));
    }
    __device__ __forceinline__ uint32_t nrow(uint64_t c, uint32_t j) const {
        return *(const uint32_t *)(base + c * block_bytes() + (uint64_t)node * sizeof(K) + (uint64_t)j * 4);
    }
    __device__ __forceinline__ K key(uint64_t s) const {
        if (node == 1) return nkey(s, 0);
        const uint64_t c = s / node;
        return nkey(c, (uint32_t)(s - c * node));
    }
    __device__ __forceinline__ uint32_t row(uint64_t s) const {
        if (node == 1) return nrow(s, 0);
        const uint64_t c = s / node;
        return nrow(c, (uint32_t)(s - c * node));
    }
    __device__ __forceinline__ const K *node_ptr(uint64_t c) const { return (const K *)(base + c * block_bytes()); }
};

template <typename K, bool AOS>
struct Store;

template <typename K>
struct Store<K, false> {
    K *__restrict__ k;
    uint32_t *__restrict__ r;
    uint32_t node;
    __device__ __forceinline__ void put(uint64_t s, K key, uint32_t row) const {
        k[s] = key;
        r[s] = row;
    }
};

template <typename K>
struct Store<K, true> {
    char *__restrict__ base;
    uint32_t *r_unused;
    uint32_t node;
    uint32_t stride;
    __device__ __forceinline__ void put(uint64_t s, K key, uint32_t row) const {
        const uint64_t c = node == 1 ? s : s / node;
        const uint32_t j = (uint32_t)(s - c * node);
        char *blk = base + c * (uint64_t)stride;
        store_key_words<K>(blk + (uint64_t)j * sizeof(K), key);
        *(uint32_t *)(blk + (uint64_t)node * sizeof(K) + (uint64_t)j * 4) = row;
    }
};

template <typename K, bool AOS>
inline Load<K, AOS> make_load(const idx_index *h) {
    Load<K, AOS> L{};
    if constexpr (AOS) {
        L.base = (const char *)h->keys;
        L.r_unused = nullptr;
        L.stride = h->stride;
    } else {
        L.k = (const K *)h->keys;
        L.r = h->rowids;
    }
    L.node = h->node;
    return L;
}

template <typename K, bool AOS>
inline Store<K, AOS> make_store(idx_index *h) {
    Store<K, AOS> S{};
    if constexpr (AOS) {
        S.base = (char *)h->keys;
        S.r_unused = nullptr;
        S.stride = h->stride;
    } else {
        S.k = (K *)h->keys;
        S.r = h->rowids;
    }
    S.node = h->node;
    return S;
}

template <typename K>
__device__ __forceinline__ K key_max() {
    return ~K(0);
}

}  // namespace idx
