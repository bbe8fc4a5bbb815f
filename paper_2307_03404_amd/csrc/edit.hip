// Dynamic-grid edits: coarse-to-fine growth and pruning (Sec. 6.1: the map is
// a dynamic voxel grid that grows to a peak of 512^3).
//
// Both edits are stream compactions: a flag per item, an exclusive prefix
// count that numbers the flagged items in order, and a write pass.  Flags are
// packed 32 to a word; a chunk is EDIT_WORDS words (one workgroup), and the
// count takes three steps:
//   flag kernel   the chunk's words, the exclusive prefix of each word's
//                 popcount inside the chunk, and the chunk's total;
//   k_scan_chunks one workgroup turns the chunk totals into exclusive chunk
//                 offsets and writes the grand total to the caller's n_out;
//   write pass    flagged item i gets id = chunk offset + word prefix +
//                 popcount of the lower bits of its word.
//
// Growth.  R vertices per axis become 2R - 1: fine vertex 2v is coarse vertex
// v, voxel size halves, the origin stays.  A fine vertex is allocated when a
// coarse cell whose closed box holds it has an allocated corner; records are
// numbered in lattice order.  Along an axis, fine coordinate 2v lies in the
// cells of coarse vertices v-1 .. v+1 (clipped to the lattice) and 2v+1 in
// those of v .. v+1, so the flag is an OR over that box of coarse vertices.
// It is evaluated bit-parallel: the coarse allocation bits of each (x, y)
// row, OR-ed over the 1-3 x 1-3 neighbouring rows, then dilated along z by
// shifts.  The compaction runs over fine rows padded to whole words.
// A fine record is the coarse trilinear interpolant at its vertex, density
// halved (density is per voxel, so each world-length step keeps its optical
// depth): 1, 2, 4 or 8 coarse records with exact power-of-two weights,
// summed in FP64 in corner order and rounded once to FP32.
//
// Pruning.  Records with density <= tau are dropped, the others keep their
// order and get new ids, and the link table is rewritten (dropped -> -1).
#include "internal.hpp"

namespace pxm {

namespace {

constexpr int EDIT_THREADS = 256;
constexpr int EDIT_WORDS = EDIT_CHUNK / 32;             // words per chunk, one per thread
constexpr int KEEP_ITERS = EDIT_CHUNK / EDIT_THREADS;   // records per thread in the prune flags
constexpr int SCAN_THREADS = 1024;
constexpr int LINK_PER_THREAD = 8;
constexpr int LINK_ITEMS = LINK_PER_THREAD * EDIT_THREADS;   // link-table items per workgroup pass
constexpr int UNIT_BATCHES = 4;                         // 8-vertex batches a wave requests at once
static_assert(EDIT_WORDS == EDIT_THREADS, "one thread per flag word of a chunk");

__device__ __forceinline__ bool link_ok(int32_t l, int64_t n) { return (uint32_t)l < (uint64_t)n; }

// Exclusive prefix of `v` over the workgroup's threads; `total` gets the sum.
__device__ __forceinline__ int block_exclusive(int v, int& total) {
    __shared__ int s_wave[EDIT_THREADS / WAVE];
    const int lane = lane_id(), w = threadIdx.x / WAVE;
    int incl = v;
    for (int d = 1; d < WAVE; d <<= 1) {
        const int o = __shfl_up(incl, d, WAVE);
        if (lane >= d) incl += o;
    }
    if (lane == WAVE - 1) s_wave[w] = incl;
    __syncthreads();
    int before = 0;
    total = 0;
#pragma unroll
    for (int i = 0; i < EDIT_THREADS / WAVE; ++i) {
        before += i < w ? s_wave[i] : 0;
        total += s_wave[i];
    }
    return before + incl - v;
}

// Chunk epilogue: thread t owns word t of the chunk.
__device__ __forceinline__ void finish_chunk(uint32_t bits, int64_t gw, int64_t nw, uint32_t* words, int32_t* wpre,
                                             int32_t* chunk_total) {
    const int cnt = __popc(bits);
    int total;
    const int pre = block_exclusive(cnt, total);
    if (gw < nw) {
        words[gw] = bits;
        wpre[gw] = pre;
    }
    if (threadIdx.x == 0) chunk_total[blockIdx.x] = total;
}

// ---------------------------------------------------------------- pruning

// Record r survives iff its density exceeds tau.  Pass `it` of wave w covers
// 64 consecutive records, i.e. words 8 it + 2w and 8 it + 2w + 1 of the chunk.
__global__ __launch_bounds__(EDIT_THREADS) void k_keep_flags(const float* __restrict__ data, int S, float tau, int64_t n,
                                                             uint32_t* __restrict__ words, int32_t* __restrict__ wpre,
                                                             int32_t* __restrict__ chunk_total) {
    __shared__ uint32_t s_words[EDIT_WORDS];
    const int64_t base = (int64_t)blockIdx.x * EDIT_CHUNK;
    const int lane = lane_id(), w = threadIdx.x / WAVE;
    for (int it = 0; it < KEEP_ITERS; ++it) {
        const int64_t r = base + it * EDIT_THREADS + threadIdx.x;
        const bool f = r < n && data[r * S] > tau;
        const unsigned long long m = __ballot(f);
        if (lane == 0) s_words[it * 8 + 2 * w] = (uint32_t)m;
        if (lane == 32) s_words[it * 8 + 2 * w + 1] = (uint32_t)(m >> 32);
    }
    __syncthreads();
    finish_chunk(s_words[threadIdx.x], (int64_t)blockIdx.x * EDIT_WORDS + threadIdx.x, (n + 31) / 32, words, wpre,
                 chunk_total);
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

// id of item i among the flagged ones, or -1.
__device__ __forceinline__ int32_t compact_id(const uint32_t* words, const int32_t* wpre,
                                              const int32_t* chunk_off, int64_t i) {
    const int64_t w = i >> 5;
    const uint32_t bits = words[w];
    const int b = (int)(i & 31);
    if (!((bits >> b) & 1u)) return -1;
    return chunk_off[w / EDIT_WORDS] + wpre[w] + __popc(bits & ((1u << b) - 1u));
}

// 8 lanes per record: lanes p < S/4 copy float4 p of it (at most 7), lane 7
// writes its remap entry.
__global__ __launch_bounds__(EDIT_THREADS) void k_prune_copy(const float* __restrict__ data, int S, int64_t n,
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
        } else if (id >= 0 && part < S / 4) {
            reinterpret_cast<float4*>(out + (int64_t)id * S)[part] =
                reinterpret_cast<const float4*>(data + r * S)[part];
        }
    }
}

__global__ __launch_bounds__(EDIT_THREADS) void k_relink(const int32_t* link, int64_t nv, int64_t n_alloc,
                                                         const int32_t* __restrict__ remap, int32_t* link_out) {
    const int64_t stride = (int64_t)gridDim.x * LINK_ITEMS;
    for (int64_t v0 = (int64_t)blockIdx.x * LINK_ITEMS; v0 < nv; v0 += stride) {
        int32_t l[LINK_PER_THREAD];
#pragma unroll
        for (int k = 0; k < LINK_PER_THREAD; ++k) {
            const int64_t v = v0 + k * EDIT_THREADS + threadIdx.x;
            l[k] = v < nv ? link[v] : -1;
        }
#pragma unroll
        for (int k = 0; k < LINK_PER_THREAD; ++k) l[k] = link_ok(l[k], n_alloc) ? remap[l[k]] : -1;
#pragma unroll
        for (int k = 0; k < LINK_PER_THREAD; ++k) {
            const int64_t v = v0 + k * EDIT_THREADS + threadIdx.x;
            if (v < nv) link_out[v] = l[k];
        }
    }
}

// ---------------------------------------------------------------- growth

struct Lattice {
    int R[3];     // coarse vertices per axis
    int Rf[3];    // fine vertices per axis, 2R - 1
    int WC;       // coarse allocation words per (x, y) row
    int WF;       // fine flag words per (x, y) row
};

// Coarse allocation bits, rows padded to WC words: one lane per padded item,
// a ballot per 64.  The loop runs over a multiple of 64 items so every wave
// reaches the ballot whole.
__global__ __launch_bounds__(EDIT_THREADS) void k_coarse_bits(KGrid g, Lattice L, int64_t n_items,
                                                              uint32_t* __restrict__ vbits) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t padded = (n_items + WAVE - 1) / WAVE * WAVE;
    const int lane = lane_id();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < padded; i += stride) {
        bool f = false;
        if (i < n_items) {
            const uint32_t w = (uint32_t)(i >> 5);
            const uint32_t row = w / (uint32_t)L.WC;
            const int z = (int)(w - row * (uint32_t)L.WC) * 32 + (int)(i & 31);
            f = z < L.R[2] && link_ok(g.link[(int64_t)row * L.R[2] + z], g.n_alloc);
        }
        const unsigned long long m = __ballot(f);
        const int64_t w0 = (i - lane) >> 5;
        if (lane == 0 && w0 * 32 < n_items) vbits[w0] = (uint32_t)m;
        if (lane == 32 && (w0 + 1) * 32 < n_items) vbits[w0 + 1] = (uint32_t)(m >> 32);
    }
}

// 64 coarse bits of row `row` starting at coarse z = p (p >= -1; bits outside
// the lattice read 0).
__device__ __forceinline__ uint64_t coarse_window(const uint32_t* vbits, int64_t row, int WC, int p) {
    const uint32_t* r = vbits + row * WC;
    if (p < 0) {
        const uint64_t v = (uint64_t)r[0] | ((WC > 1 ? (uint64_t)r[1] : 0ull) << 32);
        return v << 1;
    }
    const int wi = p >> 5, sh = p & 31;
    const uint64_t lo = wi < WC ? r[wi] : 0u, hi = wi + 1 < WC ? r[wi + 1] : 0u;
    return (lo | (hi << 32)) >> sh;
}

// One thread per fine flag word: fine row (fx, fy), fine z in [32 l, 32 l + 32).
// Window bit k is coarse z = 16 l - 1 + k; fine z = 32 l + j sits on or after
// coarse vertex 16 l + (j >> 1), window bit (j >> 1) + 1.
__global__ __launch_bounds__(EDIT_THREADS) void k_grow_flags(const uint32_t* __restrict__ vbits, Lattice L, int64_t nw,
                                                             uint32_t* __restrict__ words, int32_t* __restrict__ wpre,
                                                             int32_t* __restrict__ chunk_total) {
    const int64_t gw = (int64_t)blockIdx.x * EDIT_WORDS + threadIdx.x;
    uint32_t bits = 0;
    if (gw < nw) {
        const uint32_t row = (uint32_t)(gw / L.WF);
        const int l = (int)(gw - (int64_t)row * L.WF);
        const int fx = (int)(row / (uint32_t)L.Rf[1]), fy = (int)(row - (uint32_t)fx * L.Rf[1]);
        const int vx = fx >> 1, vy = fy >> 1;
        const int x0 = (fx & 1) ? vx : max(vx - 1, 0), x1 = (fx & 1) ? vx + 1 : min(vx + 1, L.R[0] - 1);
        const int y0 = (fy & 1) ? vy : max(vy - 1, 0), y1 = (fy & 1) ? vy + 1 : min(vy + 1, L.R[1] - 1);
        uint64_t W = 0;
        for (int x = x0; x <= x1; ++x)
            for (int y = y0; y <= y1; ++y) W |= coarse_window(vbits, (int64_t)x * L.R[1] + y, L.WC, 16 * l - 1);
        const uint64_t D2 = W | (W >> 1);     // bit k: coarse k or k+1   (odd fine z)
        const uint64_t D3 = D2 | (W << 1);    // bit k: coarse k-1 .. k+1 (even fine z)
        const int jend = min(32, L.Rf[2] - 32 * l);
        for (int j = 0; j < jend; ++j) {
            const int k = (j >> 1) + 1;
            bits |= (uint32_t)((((j & 1) ? D2 : D3) >> k) & 1ull) << j;
        }
    }
    finish_chunk(bits, gw, nw, words, wpre, chunk_total);
}

// One lane per padded fine item; items past the row's end are padding.  A
// thread takes LINK_PER_THREAD items and issues all their loads first.
__global__ __launch_bounds__(EDIT_THREADS) void k_fine_link(Lattice L, int64_t n_items,
                                                            const uint32_t* __restrict__ words,
                                                            const int32_t* __restrict__ wpre,
                                                            const int32_t* __restrict__ chunk_off,
                                                            int32_t* __restrict__ link_fine) {
    // neighbouring passes share cache lines of link_fine: keep them on one XCD
    const int64_t stride = (int64_t)gridDim.x * LINK_ITEMS;
    for (int64_t i0 = xcd_tile(blockIdx.x, gridDim.x) * LINK_ITEMS; i0 < n_items; i0 += stride) {
        uint32_t bits[LINK_PER_THREAD];
        int32_t base[LINK_PER_THREAD];
#pragma unroll
        for (int k = 0; k < LINK_PER_THREAD; ++k) {
            const int64_t i = i0 + k * EDIT_THREADS + threadIdx.x;
            bits[k] = 0u;
            base[k] = 0;
            if (i < n_items) {
                const int64_t w = i >> 5;
                bits[k] = words[w];
                base[k] = chunk_off[w / EDIT_WORDS] + wpre[w];
            }
        }
#pragma unroll
        for (int k = 0; k < LINK_PER_THREAD; ++k) {
            const int64_t i = i0 + k * EDIT_THREADS + threadIdx.x;
            const uint32_t w = (uint32_t)(i >> 5);
            const uint32_t row = w / (uint32_t)L.WF;
            const int fz = (int)(w - row * (uint32_t)L.WF) * 32 + (int)(i & 31);
            const int b = (int)(i & 31);
            if (i < n_items && fz < L.Rf[2])
                link_fine[(int64_t)row * L.Rf[2] + fz] =
                    ((bits[k] >> b) & 1u) ? base[k] + __popc(bits[k] & ((1u << b) - 1u)) : -1;
        }
    }
}

// Records by coarse vertex: coarse vertex v owns the fine vertices
// 2v + o, o in {0,1}^3, and all eight interpolate from the corners v + o' of
// coarse cell v (o' a subset of o's bits; weight 1/2 per odd axis).  A group
// of 8 lanes takes one v: lane k first fetches corner link v + o_k and the id
// of fine vertex 2v + o_k, for UNIT_BATCHES batches of 8 vertices at once;
// then, per batch with an allocated fine vertex, lane p < S/4 (7 at SH degree
// 2) fetches float4 p of the 8 corner records and writes float4 p of each
// allocated fine record.
// Sums run over corners in (x, y, z) bit order in FP64.
__global__ __launch_bounds__(EDIT_THREADS) void k_fine_data(KGrid g, Lattice L, const int32_t* __restrict__ link_fine,
                                                            int64_t n_fine, float* __restrict__ out) {
    const int lane = lane_id(), k = lane & 7, gbase = lane & ~7;
    const int64_t nc = (int64_t)L.R[0] * L.R[1] * L.R[2];
    const int64_t waves = (int64_t)gridDim.x * (EDIT_THREADS / WAVE);
    const float4* data4 = reinterpret_cast<const float4*>(g.data);
    const int S = record_floats(g.deg), Q = S / 4;   // float4 parts per record (at most 7)
    // neighbouring units write records that share cache lines: keep them on one XCD
    const int64_t first = xcd_tile(blockIdx.x, gridDim.x) * (EDIT_THREADS / WAVE) + threadIdx.x / WAVE;
    for (int64_t s = first; s * 8 * UNIT_BATCHES < nc; s += waves) {
        int32_t lids[UNIT_BATCHES], fids[UNIT_BATCHES];
#pragma unroll
        for (int j = 0; j < UNIT_BATCHES; ++j) {
            const int64_t u = (s * UNIT_BATCHES + j) * 8 + (lane >> 3);
            lids[j] = fids[j] = -1;
            if (u < nc) {
                const uint32_t r = (uint32_t)u / (uint32_t)L.R[2];   // u < R^3 < 2^31 / 8
                const int vz = (int)((uint32_t)u - r * (uint32_t)L.R[2]);
                const int vx = (int)(r / (uint32_t)L.R[1]), vy = (int)(r - (uint32_t)vx * L.R[1]);
                const int ox = (k >> 2) & 1, oy = (k >> 1) & 1, oz = k & 1;
                if (vx + ox < L.R[0] && vy + oy < L.R[1] && vz + oz < L.R[2]) {
                    lids[j] = g.link[(int64_t)(vx + ox) * g.sx + (int64_t)(vy + oy) * g.sy + (vz + oz)];
                    fids[j] = link_fine[((int64_t)(2 * vx + ox) * L.Rf[1] + (2 * vy + oy)) * L.Rf[2] + (2 * vz + oz)];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < UNIT_BATCHES; ++j) {
            const int32_t lid = lids[j], fid = fids[j];
            if (__ballot(link_ok(fid, n_fine)) == 0ull) continue;
            const int p = k;   // float4 part handled by this lane (none when p >= Q)
            float4 v[8];
            bool ok[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int32_t lb = __shfl(lid, gbase + b, WAVE);
                ok[b] = link_ok(lb, g.n_alloc);
                v[b] = (ok[b] && p < Q) ? data4[(int64_t)lb * Q + p] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const int32_t fo = __shfl(fid, gbase + o, WAVE);
                if (!link_ok(fo, n_fine) || p >= Q) continue;
                const double wt = 1.0 / (double)(1 << __popc(o));
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    if ((b & ~o) || !ok[b]) continue;
                    a0 += wt * (double)v[b].x;
                    a1 += wt * (double)v[b].y;
                    a2 += wt * (double)v[b].z;
                    a3 += wt * (double)v[b].w;
                }
                if (p == 0) a0 *= 0.5;
                reinterpret_cast<float4*>(out + (int64_t)fo * S)[p] =
                    make_float4((float)a0, (float)a1, (float)a2, (float)a3);
            }
        }
    }
}

unsigned stride_blocks(int64_t items, int per_block = EDIT_THREADS) {
    const int64_t b = (items + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : b > (1 << 20) ? (1 << 20) : b);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Lattice lattice(const KGrid& g) {
    Lattice L;
    for (int a = 0; a < 3; ++a) {
        L.R[a] = g.R[a];
        L.Rf[a] = 2 * g.R[a] - 1;
    }
    L.WC = (L.R[2] + 31) / 32;
    L.WF = (L.Rf[2] + 31) / 32;
    return L;
}

// Workspace of a compaction over nw flag words: words, word prefixes, chunk
// totals (then offsets), each 256-byte aligned.
struct Compaction {
    uint32_t* words;
    int32_t* wpre;
    int32_t* chunk;
    int64_t n_chunks;
};

size_t compaction_words_bytes(int64_t nw) {
    return 2 * align256(nw * 4) + align256((nw + EDIT_WORDS - 1) / EDIT_WORDS * 4);
}

Compaction carve(void* ws, int64_t nw) {
    char* p = static_cast<char*>(ws);
    Compaction c;
    c.words = reinterpret_cast<uint32_t*>(p);
    c.wpre = reinterpret_cast<int32_t*>(p + align256(nw * 4));
    c.chunk = reinterpret_cast<int32_t*>(p + 2 * align256(nw * 4));
    c.n_chunks = (nw + EDIT_WORDS - 1) / EDIT_WORDS;
    return c;
}

hipError_t scan(const Compaction& c, int64_t* n_out, hipStream_t st) {
    hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(SCAN_THREADS), 0, st, c.chunk, c.n_chunks, n_out);
    return hipGetLastError();
}

}  // namespace

size_t prune_workspace_bytes(int64_t n_alloc) { return compaction_words_bytes((n_alloc + 31) / 32) + 4 * n_alloc; }

size_t grow_workspace_bytes(const int R[3]) {
    const int64_t rows_c = (int64_t)R[0] * R[1], rows_f = (int64_t)(2 * R[0] - 1) * (2 * R[1] - 1);
    const int64_t wc = (R[2] + 31) / 32, wf = (2 * R[2] - 1 + 31) / 32;
    return align256(rows_c * wc * 4) + compaction_words_bytes(rows_f * wf);
}

hipError_t launch_upsample_link(const KGrid& g, int32_t* link_fine, int64_t* n_fine, void* ws, hipStream_t st) {
    const Lattice L = lattice(g);
    const int64_t rows_c = (int64_t)L.R[0] * L.R[1], rows_f = (int64_t)L.Rf[0] * L.Rf[1];
    uint32_t* vbits = static_cast<uint32_t*>(ws);
    const int64_t n_coarse_items = rows_c * L.WC * 32, nw = rows_f * L.WF;
    const Compaction c = carve(static_cast<char*>(ws) + align256(rows_c * L.WC * 4), nw);
    hipLaunchKernelGGL(k_coarse_bits, dim3(stride_blocks(n_coarse_items)), dim3(EDIT_THREADS), 0, st, g, L,
                       n_coarse_items, vbits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grow_flags, dim3((unsigned)c.n_chunks), dim3(EDIT_THREADS), 0, st, vbits, L, nw, c.words,
                       c.wpre, c.chunk);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan(c, n_fine, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_fine_link, dim3(stride_blocks(nw * 32, LINK_ITEMS)), dim3(EDIT_THREADS), 0, st, L, nw * 32, c.words,
                       c.wpre, c.chunk, link_fine);
    return hipGetLastError();
}

hipError_t launch_upsample_data(const KGrid& g, const int32_t* link_fine, int64_t n_fine, float* data_fine,
                                hipStream_t st) {
    const Lattice L = lattice(g);
    const int64_t units = (int64_t)L.R[0] * L.R[1] * L.R[2];   // coarse vertices, 8 lanes each
    hipLaunchKernelGGL(k_fine_data, dim3(stride_blocks(units * 8, EDIT_THREADS * UNIT_BATCHES)), dim3(EDIT_THREADS), 0, st, g, L, link_fine, n_fine,
                       data_fine);
    return hipGetLastError();
}

hipError_t launch_prune(const KGrid& g, float tau, int32_t* link_out, float* data_out, int64_t* n_out, void* ws,
                        hipStream_t st) {
    const int64_t n = g.n_alloc, nv = (int64_t)g.R[0] * g.R[1] * g.R[2], nw = (n + 31) / 32;
    const Compaction c = carve(ws, nw);
    int32_t* remap = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + compaction_words_bytes(nw));
    hipError_t e;
    if (c.n_chunks > 0) {
        hipLaunchKernelGGL(k_keep_flags, dim3((unsigned)c.n_chunks), dim3(EDIT_THREADS), 0, st, g.data,
                           record_floats(g.deg), tau, n, c.words,
                           c.wpre, c.chunk);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = scan(c, n_out, st)) != hipSuccess) return e;
    if (n > 0) {
        hipLaunchKernelGGL(k_prune_copy, dim3(stride_blocks(n * 8)), dim3(EDIT_THREADS), 0, st, g.data,
                           record_floats(g.deg), n, c.words,
                           c.wpre, c.chunk, remap, data_out);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_relink, dim3(stride_blocks(nv, LINK_ITEMS)), dim3(EDIT_THREADS), 0, st, g.link, nv, n, remap, link_out);
    return hipGetLastError();
}

}  // namespace pxm
