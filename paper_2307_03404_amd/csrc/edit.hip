// Dynamic-grid edits: coarse-to-fine growth and pruning (Sec. 5: the map is
// a dynamic voxel grid that grows to a peak of 512^3).
//
// Both edits are stream compactions: a flag per item (a fine lattice vertex,
// or a record), an exclusive prefix count that numbers the flagged items in
// order, and a write pass.  The count runs in three launches over chunks of
// EDIT_CHUNK items:
//   k_flags       one ballot per 64 items -> flag words; per chunk, the
//                 exclusive prefix of each word inside the chunk and the
//                 chunk's total;
//   k_scan_chunks one workgroup turns the chunk totals into exclusive chunk
//                 offsets and writes the grand total to the caller's n_out;
//   write pass    item e, if flagged, gets id = chunk offset + word prefix +
//                 popcount of the lower bits of its word.
//
// Growth.  R vertices per axis become 2R - 1: fine vertex 2v is coarse vertex
// v, voxel size halves, the origin stays.  A fine vertex is allocated when a
// coarse cell whose closed box holds it has an allocated corner; records are
// numbered in lattice order.  Its record is the coarse trilinear interpolant
// at its position, with the density halved (density is per voxel, so each
// world-length step keeps its optical depth).  Along an axis the fine vertex
// sits on a coarse vertex (weight 1) or halfway between two (weights 1/2), so
// a record mixes 1, 2, 4 or 8 coarse records with exact power-of-two weights,
// summed in FP64 in corner order and rounded once to FP32.
//
// Pruning.  Records with density <= tau are dropped, the others keep their
// order and get new ids, and the link table is rewritten (dropped -> -1).
#include "internal.hpp"

namespace pxm {

namespace {

constexpr int EDIT_THREADS = 256;
constexpr int EDIT_ITERS = EDIT_CHUNK / EDIT_THREADS;   // items per thread in k_flags
constexpr int SCAN_THREADS = 1024;
static_assert(EDIT_CHUNK / 32 == WAVE, "one wave scans the flag words of a chunk");

__device__ __forceinline__ bool link_ok(int32_t l, int64_t n) { return (uint32_t)l < (uint64_t)n; }

// Fine vertex e of the (2R-1)^3 lattice: allocated iff some coarse vertex in
// the box spanned by the coarse cells holding it is allocated.
struct FineFlag {
    const int32_t* link;
    int64_t n_alloc;
    int R[3];      // coarse vertices per axis
    int Rf[3];     // fine vertices per axis
    __device__ bool operator()(int64_t e) const {
        const int fz = (int)(e % Rf[2]);
        const int64_t r = e / Rf[2];
        const int fy = (int)(r % Rf[1]);
        const int fx = (int)(r / Rf[1]);
        int lo[3], hi[3];
        const int f[3] = {fx, fy, fz};
        for (int a = 0; a < 3; ++a) {
            const int v = f[a] >> 1;
            if (f[a] & 1) {
                lo[a] = v;
                hi[a] = v + 1;
            } else {
                lo[a] = max(v - 1, 0);
                hi[a] = min(v + 1, R[a] - 1);
            }
        }
        const int64_t sy = R[2], sx = (int64_t)R[1] * R[2];
        for (int x = lo[0]; x <= hi[0]; ++x)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int z = lo[2]; z <= hi[2]; ++z)
                    if (link_ok(link[x * sx + y * sy + z], n_alloc)) return true;
        return false;
    }
};

// Record r survives pruning iff its density exceeds tau.
struct KeepFlag {
    const float* data;
    float tau;
    __device__ bool operator()(int64_t r) const { return data[r * REC] > tau; }
};

// Chunk b covers items [b*EDIT_CHUNK, (b+1)*EDIT_CHUNK).  Pass `it` of wave w
// covers 64 consecutive items, i.e. words it*8 + 2w and it*8 + 2w + 1 of the
// chunk's 64 words.
template <typename Flag>
__global__ __launch_bounds__(EDIT_THREADS) void k_flags(Flag flag, int64_t n, uint32_t* __restrict__ words,
                                                        int32_t* __restrict__ wpre, int32_t* __restrict__ chunk_total) {
    __shared__ uint32_t s_words[EDIT_CHUNK / 32];
    const int64_t base = (int64_t)blockIdx.x * EDIT_CHUNK;
    const int lane = lane_id(), w = threadIdx.x / WAVE;
    for (int it = 0; it < EDIT_ITERS; ++it) {
        const int64_t e = base + it * EDIT_THREADS + threadIdx.x;
        const bool f = e < n && flag(e);
        const unsigned long long m = __ballot(f);
        if (lane == 0) s_words[it * 8 + 2 * w] = (uint32_t)m;
        if (lane == 32) s_words[it * 8 + 2 * w + 1] = (uint32_t)(m >> 32);
    }
    __syncthreads();
    if (threadIdx.x < WAVE) {
        const uint32_t bits = s_words[threadIdx.x];
        const int cnt = __popc(bits);
        int incl = cnt;
        for (int d = 1; d < WAVE; d <<= 1) {
            const int o = __shfl_up(incl, d, WAVE);
            if (lane >= d) incl += o;
        }
        const int64_t gw = (int64_t)blockIdx.x * (EDIT_CHUNK / 32) + threadIdx.x;
        if (gw < (n + 31) / 32) {
            words[gw] = bits;
            wpre[gw] = incl - cnt;
        }
        if (lane == WAVE - 1) chunk_total[blockIdx.x] = incl;
    }
}

// One workgroup: exclusive scan of the chunk totals in place; *n_out = sum.
// Thread t owns a contiguous run of ceil(nc / SCAN_THREADS) totals.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_chunks(int32_t* __restrict__ chunk, int64_t nc,
                                                              int64_t* __restrict__ n_out) {
    __shared__ int64_t s_wave[SCAN_THREADS / WAVE];
    const int64_t per = (nc + SCAN_THREADS - 1) / SCAN_THREADS;
    const int64_t b0 = min((int64_t)threadIdx.x * per, nc), b1 = min(b0 + per, nc);
    int64_t sum = 0;
    for (int64_t b = b0; b < b1; ++b) sum += chunk[b];
    // inclusive scan of the per-thread sums: within waves, then across them
    const int lane = lane_id(), w = threadIdx.x / WAVE;
    int64_t incl = sum;
    for (int d = 1; d < WAVE; d <<= 1) {
        const int64_t o = __shfl_up(incl, d, WAVE);
        if (lane >= d) incl += o;
    }
    if (lane == WAVE - 1) s_wave[w] = incl;
    __syncthreads();
    int64_t before = 0;
    for (int i = 0; i < w; ++i) before += s_wave[i];
    int64_t run = before + incl - sum;
    for (int64_t b = b0; b < b1; ++b) {
        const int32_t c = chunk[b];
        chunk[b] = (int32_t)run;
        run += c;
    }
    if (threadIdx.x == SCAN_THREADS - 1) *n_out = before + incl;
}

// id of item e among the flagged ones, or -1.
__device__ __forceinline__ int32_t compact_id(const uint32_t* words, const int32_t* wpre,
                                              const int32_t* chunk_off, int64_t e) {
    const int64_t w = e >> 5;
    const uint32_t bits = words[w];
    const int b = (int)(e & 31);
    if (!((bits >> b) & 1u)) return -1;
    return chunk_off[w / (EDIT_CHUNK / 32)] + wpre[w] + __popc(bits & ((1u << b) - 1u));
}

__global__ __launch_bounds__(EDIT_THREADS) void k_fine_link(int64_t nf, const uint32_t* __restrict__ words,
                                                            const int32_t* __restrict__ wpre,
                                                            const int32_t* __restrict__ chunk_off,
                                                            int32_t* __restrict__ link_fine) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += stride)
        link_fine[e] = compact_id(words, wpre, chunk_off, e);
}

// One lane per fine vertex; allocated ones gather their 1-8 coarse records.
__global__ __launch_bounds__(EDIT_THREADS) void k_fine_data(KGrid g, int Rf1, int Rf2, int64_t nf,
                                                            const int32_t* __restrict__ link_fine,
                                                            int64_t n_fine, float* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += stride) {
        const int32_t id = link_fine[e];
        if (!link_ok(id, n_fine)) continue;
        const int fz = (int)(e % Rf2);
        const int64_t r = e / Rf2;
        const int fy = (int)(r % Rf1), fx = (int)(r / Rf1);
        const int odd = ((fx & 1) << 2) | ((fy & 1) << 1) | (fz & 1);
        const int64_t c0 = (int64_t)(fx >> 1) * g.sx + (int64_t)(fy >> 1) * g.sy + (fz >> 1);
        const double wt = 1.0 / (double)(1 << __popc(odd));
        double acc[REC];
#pragma unroll
        for (int j = 0; j < REC; ++j) acc[j] = 0.0;
        // corners in (x, y, z) bit order; a corner offset along an even axis has weight 0
        for (int b = 0; b < 8; ++b) {
            if (b & ~odd) continue;
            const int32_t l = g.link[c0 + ((b >> 2) & 1) * g.sx + ((b >> 1) & 1) * g.sy + (b & 1)];
            if (!link_ok(l, g.n_alloc)) continue;
            const float4* src = reinterpret_cast<const float4*>(g.data + (int64_t)l * REC);
#pragma unroll
            for (int q = 0; q < REC / 4; ++q) {
                const float4 v = src[q];
                acc[4 * q + 0] += wt * (double)v.x;
                acc[4 * q + 1] += wt * (double)v.y;
                acc[4 * q + 2] += wt * (double)v.z;
                acc[4 * q + 3] += wt * (double)v.w;
            }
        }
        acc[0] *= 0.5;
        float4* dst = reinterpret_cast<float4*>(out + (int64_t)id * REC);
#pragma unroll
        for (int q = 0; q < REC / 4; ++q)
            dst[q] = make_float4((float)acc[4 * q], (float)acc[4 * q + 1], (float)acc[4 * q + 2],
                                 (float)acc[4 * q + 3]);
    }
}

// 8 lanes per record (7 carry a float4): new id, remap entry, copy.
__global__ __launch_bounds__(EDIT_THREADS) void k_prune_copy(const float* __restrict__ data, int64_t n,
                                                             const uint32_t* __restrict__ words,
                                                             const int32_t* __restrict__ wpre,
                                                             const int32_t* __restrict__ chunk_off,
                                                             int32_t* __restrict__ remap, float* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n * 8; t += stride) {
        const int64_t r = t >> 3;
        const int part = (int)(t & 7);
        const int32_t id = compact_id(words, wpre, chunk_off, r);
        if (part == 7) {
            remap[r] = id;
        } else if (id >= 0) {
            reinterpret_cast<float4*>(out + (int64_t)id * REC)[part] =
                reinterpret_cast<const float4*>(data + r * REC)[part];
        }
    }
}

__global__ __launch_bounds__(EDIT_THREADS) void k_relink(const int32_t* link, int64_t nv, int64_t n_alloc,
                                                         const int32_t* __restrict__ remap, int32_t* link_out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += stride) {
        const int32_t l = link[v];
        link_out[v] = link_ok(l, n_alloc) ? remap[l] : -1;
    }
}

unsigned stride_blocks(int64_t items) {
    const int64_t b = (items + EDIT_THREADS - 1) / EDIT_THREADS;
    return (unsigned)(b < 1 ? 1 : b > (1 << 20) ? (1 << 20) : b);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace carve-up for a compaction over n items: flag words, word
// prefixes, chunk totals (then offsets), each 256-byte aligned.
struct Compaction {
    uint32_t* words;
    int32_t* wpre;
    int32_t* chunk;
    int64_t n_chunks;
};

Compaction carve(void* ws, int64_t n) {
    const int64_t nw = (n + 31) / 32;
    char* p = static_cast<char*>(ws);
    Compaction c;
    c.words = reinterpret_cast<uint32_t*>(p);
    c.wpre = reinterpret_cast<int32_t*>(p + align256(nw * 4));
    c.chunk = reinterpret_cast<int32_t*>(p + 2 * align256(nw * 4));
    c.n_chunks = (n + EDIT_CHUNK - 1) / EDIT_CHUNK;
    return c;
}

template <typename Flag>
hipError_t count(const Flag& flag, int64_t n, const Compaction& c, int64_t* n_out, hipStream_t st) {
    if (c.n_chunks > 0) {
        hipLaunchKernelGGL(k_flags<Flag>, dim3((unsigned)c.n_chunks), dim3(EDIT_THREADS), 0, st, flag, n, c.words,
                           c.wpre, c.chunk);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(SCAN_THREADS), 0, st, c.chunk, c.n_chunks, n_out);
    return hipGetLastError();
}

}  // namespace

size_t compaction_bytes(int64_t n) {
    const int64_t nw = (n + 31) / 32, nc = (n + EDIT_CHUNK - 1) / EDIT_CHUNK;
    return 2 * align256(nw * 4) + align256(nc * 4);
}

hipError_t launch_upsample_link(const KGrid& g, int32_t* link_fine, int64_t* n_fine, void* ws, hipStream_t st) {
    FineFlag f;
    f.link = g.link;
    f.n_alloc = g.n_alloc;
    int64_t nf = 1;
    for (int a = 0; a < 3; ++a) {
        f.R[a] = g.R[a];
        f.Rf[a] = 2 * g.R[a] - 1;
        nf *= f.Rf[a];
    }
    const Compaction c = carve(ws, nf);
    hipError_t e = count(f, nf, c, n_fine, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fine_link, dim3(stride_blocks(nf)), dim3(EDIT_THREADS), 0, st, nf, c.words, c.wpre,
                       c.chunk, link_fine);
    return hipGetLastError();
}

hipError_t launch_upsample_data(const KGrid& g, const int32_t* link_fine, int64_t n_fine, float* data_fine,
                                hipStream_t st) {
    const int Rf0 = 2 * g.R[0] - 1, Rf1 = 2 * g.R[1] - 1, Rf2 = 2 * g.R[2] - 1;
    const int64_t nf = (int64_t)Rf0 * Rf1 * Rf2;
    hipLaunchKernelGGL(k_fine_data, dim3(stride_blocks(nf)), dim3(EDIT_THREADS), 0, st, g, Rf1, Rf2, nf, link_fine,
                       n_fine, data_fine);
    return hipGetLastError();
}

hipError_t launch_prune(const KGrid& g, float tau, int32_t* link_out, float* data_out, int64_t* n_out, void* ws,
                        hipStream_t st) {
    const int64_t n = g.n_alloc, nv = (int64_t)g.R[0] * g.R[1] * g.R[2];
    const Compaction c = carve(ws, n);
    int32_t* remap = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + compaction_bytes(n));
    KeepFlag f;
    f.data = g.data;
    f.tau = tau;
    hipError_t e = count(f, n, c, n_out, st);
    if (e != hipSuccess) return e;
    if (n > 0) {
        hipLaunchKernelGGL(k_prune_copy, dim3(stride_blocks(n * 8)), dim3(EDIT_THREADS), 0, st, g.data, n, c.words,
                           c.wpre, c.chunk, remap, data_out);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_relink, dim3(stride_blocks(nv)), dim3(EDIT_THREADS), 0, st, g.link, nv, n, remap, link_out);
    return hipGetLastError();
}

}  // namespace pxm
