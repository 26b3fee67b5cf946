// C ABI entry points of libpll (declared in include/pll.h).
#include <algorithm>
#include <new>

#include "pll_internal.h"

namespace {

constexpr int kBlock = 256;

__global__ void k_export(uint64_t total, const uint32_t* __restrict__ ent, const uint32_t* __restrict__ order,
                         uint32_t* __restrict__ hubs, uint8_t* __restrict__ dists) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t e = ent[i];
        hubs[i] = order[e >> 8];
        dists[i] = (uint8_t)(e & 255u);
    }
}

void free_index(pll_index* idx) {
    if (!idx) return;
    int cur = -1;
    bool switched = false;
    if (hipGetDevice(&cur) == hipSuccess && cur != idx->device) switched = hipSetDevice(idx->device) == hipSuccess;
    if (idx->meta) {
        if (idx->meta->refs.fetch_sub(1) == 1) {
            (void)hipFree(idx->meta->ptr);
            delete idx->meta;
        }
    } else {
        (void)hipFree(idx->d_off);
        (void)hipFree(idx->d_order);
        (void)hipFree(idx->d_lb);
    }
    if (idx->directed) {
        (void)hipFree(idx->d_off_out);
        (void)hipFree(idx->d_ent_out);
        (void)hipFree(idx->d_lb_out);
    }
    if (idx->d_bp_roots) {
        (void)hipFree(idx->d_bp_roots);
        (void)hipFree(idx->d_bp_nbrs);
        (void)hipFree(idx->d_bp_dist);
        (void)hipFree(idx->d_bp_sets);
    }
    if (idx->store) {
        if (idx->store->refs.fetch_sub(1) == 1) {
            (void)hipFree(idx->store->ptr);
            delete idx->store;
        }
    } else {
        (void)hipFree(idx->d_ent);
    }
    if (switched) (void)hipSetDevice(cur);
    delete idx;
}

}  // namespace

// Labels in the exported form from a final label array: hubs as vertex ids,
// distances as bytes (used by the allocation-free build).
int pll_export_launch(uint64_t total, const uint32_t* ent, const uint32_t* order, uint32_t* hubs, uint8_t* dists,
                      hipStream_t s) {
    if (total == 0) return PLL_OK;
    const uint64_t blocks = std::min<uint64_t>((total + kBlock - 1) / kBlock, 65536);
    k_export<<<(uint32_t)blocks, kBlock, 0, s>>>(total, ent, order, hubs, dists);
    return hipGetLastError() == hipSuccess ? PLL_OK : PLL_EDEVICE;
}

extern "C" {

int pll_build_labels(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col,
                     const uint32_t* d_order, const pll_build_opts* opts, hipStream_t stream, pll_index** out) {
    try {
        return pll_build_one(n, nnz, d_row_ptr, d_col, d_order, opts, stream, out);
    } catch (...) {
        if (out) *out = nullptr;
        return PLL_ENOMEM;
    }
}

int pll_query(const pll_index* idx, uint64_t count, const uint32_t* d_u, const uint32_t* d_v, uint32_t* d_out,
              hipStream_t stream) {
    if (!idx) return PLL_EINVAL;
    if (count && (!d_u || !d_v || !d_out)) return PLL_EINVAL;
    return pll_query_launch(idx, count, d_u, d_v, d_out, stream);
}

int pll_index_set_query_lanes(pll_index* idx, uint32_t lanes) {
    if (!idx) return PLL_EINVAL;
    if (!(lanes == 0 || lanes == 1 || lanes == 4 || lanes == 8 || lanes == 16 || lanes == 32 || lanes == 64))
        return PLL_EINVAL;
    idx->query_lanes = lanes;
    return PLL_OK;
}

int pll_index_info_get(const pll_index* idx, pll_index_info* out) {
    if (!idx || !out) return PLL_EINVAL;
    *out = idx->info;
    out->query_lanes = pll_query_lanes(idx);
    return PLL_OK;
}

int pll_export_labels_side(const pll_index* idx, uint32_t side, uint64_t* d_offsets, uint32_t* d_hubs,
                           uint8_t* d_dists, hipStream_t stream) {
    if (!idx || !d_offsets || side > PLL_LABELS_OUT) return PLL_EINVAL;
    const bool out_side = idx->directed && side == PLL_LABELS_OUT;
    const uint64_t total = out_side ? idx->total_out : idx->total;
    const uint64_t* off = out_side ? idx->d_off_out : idx->d_off;
    const uint32_t* ent = out_side ? idx->d_ent_out : idx->d_ent;
    if (total && (!d_hubs || !d_dists)) return PLL_EINVAL;
    if (hipMemcpyAsync(d_offsets, off, sizeof(uint64_t) * ((size_t)idx->n + 1), hipMemcpyDeviceToDevice, stream) !=
        hipSuccess)
        return PLL_EDEVICE;
    if (total) {
        uint64_t blocks = (total + kBlock - 1) / kBlock;
        if (blocks > 65536) blocks = 65536;
        k_export<<<(uint32_t)blocks, kBlock, 0, stream>>>(total, ent, idx->d_order, d_hubs, d_dists);
        if (hipGetLastError() != hipSuccess) return PLL_EDEVICE;
    }
    return PLL_OK;
}

int pll_export_bp(const pll_index* idx, uint32_t* d_roots, uint32_t* d_nbrs, uint8_t* d_dist, uint64_t* d_sm1,
                  uint64_t* d_s0, hipStream_t stream) {
    if (!idx) return PLL_EINVAL;
    const uint32_t t = idx->info.bp_roots;
    if (t == 0) return PLL_OK;
    if (!d_roots || !d_nbrs || !d_dist || !d_sm1 || !d_s0) return PLL_EINVAL;
    const size_t nt = (size_t)idx->n * t;
    if (hipMemcpyAsync(d_roots, idx->d_bp_roots, sizeof(uint32_t) * t, hipMemcpyDeviceToDevice, stream) !=
            hipSuccess ||
        hipMemcpyAsync(d_nbrs, idx->d_bp_nbrs, sizeof(uint32_t) * 64 * t, hipMemcpyDeviceToDevice, stream) !=
            hipSuccess ||
        hipMemcpyAsync(d_dist, idx->d_bp_dist, nt, hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return PLL_EDEVICE;
    if (nt) {
        // the (S^-1, S^0) pairs split into two arrays
        if (hipMemcpy2DAsync(d_sm1, sizeof(uint64_t), idx->d_bp_sets, sizeof(ulonglong2), sizeof(uint64_t), nt,
                             hipMemcpyDeviceToDevice, stream) != hipSuccess ||
            hipMemcpy2DAsync(d_s0, sizeof(uint64_t), reinterpret_cast<const char*>(idx->d_bp_sets) + sizeof(uint64_t),
                             sizeof(ulonglong2), sizeof(uint64_t), nt, hipMemcpyDeviceToDevice, stream) != hipSuccess)
            return PLL_EDEVICE;
    }
    return PLL_OK;
}

int pll_export_labels(const pll_index* idx, uint64_t* d_offsets, uint32_t* d_hubs, uint8_t* d_dists,
                      hipStream_t stream) {
    return pll_export_labels_side(idx, PLL_LABELS_IN, d_offsets, d_hubs, d_dists, stream);
}

int pll_build_labels_weighted(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col,
                              const uint8_t* d_w, const uint32_t* d_order, const pll_build_opts* opts,
                              hipStream_t stream, pll_index** out) {
    try {
        return pll_build_weighted(n, nnz, d_row_ptr, d_col, d_w, d_order, opts, stream, out);
    } catch (...) {
        if (out) *out = nullptr;
        return PLL_ENOMEM;
    }
}

int pll_build_labels_directed(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col,
                              const uint32_t* d_order, const pll_build_opts* opts, hipStream_t stream,
                              pll_index** out) {
    try {
        return pll_build_directed(n, nnz, d_row_ptr, d_col, d_order, opts, stream, out);
    } catch (...) {
        if (out) *out = nullptr;
        return PLL_ENOMEM;
    }
}

int pll_build_labels_batched(uint32_t count, const pll_graph_desc* graphs, const pll_build_opts* opts,
                             hipStream_t stream, pll_index** outs) {
    try {
        return pll_build_multi(count, graphs, opts, stream, outs);
    } catch (...) {
        return PLL_ENOMEM;
    }
}

void pll_index_free(pll_index* idx) {
    if (idx && idx->refs.fetch_sub(1, std::memory_order_acq_rel) == 1) free_index(idx);
}

const char* pll_status_string(int status) {
    switch (status) {
        case PLL_OK: return "ok";
        case PLL_EINVAL: return "invalid argument (malformed CSR, order not a permutation, bad option or NULL pointer)";
        case PLL_ENOMEM: return "out of memory";
        case PLL_ENOSPC: return "label arena too small; retry with a larger pll_build_opts.arena_entries";
        case PLL_EDIST: return "a shortest distance of 255 or more does not fit the uint8 labels";
        case PLL_EDEVICE: return "HIP runtime error";
        case PLL_ESCRATCH:
            return "the graph's working set or labels do not fit the fixed scratch of pll_build_labels_noalloc";
        default: return "unknown status";
    }
}

}  // extern "C"
