// Sparse TTMc, Y_(n)(i_n, :) += x * kron_{t != n} U_t(i_t, :)   (paper Alg. 2; Sec. III-C).
//
// The nonzeros of mode n are stored sorted by row (i_n) and cut into chunks of whole rows (a row
// longer than the chunk target is cut into pieces).  One wavefront walks one chunk: for each row
// segment it accumulates the Kronecker rows of its nonzeros in registers (same-row reduction
// before any global write, the accumulation over shared indices of Sec. III-C), then stores the
// finished row once.  The wave that holds the first nonzero of a row owns it and also writes the
// zero rows in the gap before it; pieces of a split row write their partial sums to a carry slot
// and a fix-up pass adds the slots in order, so the result is deterministic and Y needs no
// separate zero-fill.
//
// Kernels:
//   k_ttmc3_mfma  - order 3 with R_a, R_b <= 16.  The row sum  sum_p (x_p a_p) b_p^T  is a
//                   rank-k product over the row's nonzeros, computed 4 nonzeros at a time by
//                   v_mfma_{f32,f64}_16x16x4: lane l carries nonzero l/16 and factor column l%16.
//   k_ttmc3_lds   - the same for FP32 storage with the batch's factor rows staged in LDS tiles
//                   (and, in its residual form, the completion residuals formed inside).
//   k_ttmc3_bf    - the same for BF16 storage on v_mfma_f32_16x16x32_bf16, 32 nonzeros per
//                   instruction, the tiles column-major and x_p a_p rounded once to BF16.
//   k_ttmc_generic- any order 2..8 and K_n <= 4096 on the vector ALU; lane l owns columns l+64j.
#include "internal.h"

namespace tk {

namespace {

struct TtmcArgs {
    const int32_t* chunk_ptr;
    const int32_t* chunk_row;
    const int32_t* chunk_slot;
    int32_t nchunks;
    const int32_t* ptr;       // padded row pointers
    const int32_t* rows;
    int32_t S;
    int32_t In;
    const int32_t* idx;       // [nm1][nnz] padded stream; bit 31 of idx[0] flags the first entry of a row
    int64_t nnz;              // padded stream length
    const void* val;
    const void* F[kMaxOrder - 1];
    int32_t ld[kMaxOrder - 1];
    int32_t R[kMaxOrder - 1];
    int32_t nm1;
    int32_t K;
    void* Y;
    void* carry;
};

template <typename ST> __device__ inline float ld_f32(const void* p, int64_t i);
template <> __device__ inline float ld_f32<float>(const void* p, int64_t i) { return ((const float*)p)[i]; }
template <> __device__ inline float ld_f32<bf16_t>(const void* p, int64_t i) { return bf16_to_f32(((const bf16_t*)p)[i]); }

template <typename AT, typename ST>
__device__ inline AT load_as(const void* p, int64_t i) {
    if constexpr (sizeof(AT) == 8) return ((const double*)p)[i];
    else return ld_f32<ST>(p, i);
}
template <typename AT, typename ST>
__device__ inline AT load_as(const ST* p, int64_t i) {
    return load_as<AT, ST>((const void*)p, i);
}
template <typename AT, typename ST>
__device__ inline AT load_as(const ST* p, uint32_t i) {
    if constexpr (sizeof(AT) == 8) return ((const double*)p)[i];
    else if constexpr (sizeof(ST) == 4) return ((const float*)p)[i];
    else return bf16_to_f32(((const bf16_t*)p)[i]);
}

// Read-only layout arrays indexed by a wave-uniform value: reading through the constant address
// space lets the compiler use scalar loads (tracked apart from the vector-memory counter).
__device__ inline int32_t ld_const(const int32_t* p, int64_t i) {
    return ((const __attribute__((address_space(4))) int32_t*)p)[i];
}

// Zero the rows of Y strictly between the previous non-empty row and row s (and, for the last
// non-empty row, every row after it).  Called by the owner of row s, once per row.
template <typename AT>
__device__ inline void zero_gaps(const TtmcArgs& a, int s, int lane) {
    AT* Y = (AT*)a.Y;
    int g0 = (s == 0) ? 0 : ld_const(a.rows, s - 1) + 1;
    int g1 = ld_const(a.rows, s);
    int64_t K = a.K;
    for (int64_t e = (int64_t)g0 * K + lane; e < (int64_t)g1 * K; e += 64) Y[e] = AT(0);
    if (s == a.S - 1)
        for (int64_t e = (int64_t)(g1 + 1) * K + lane; e < (int64_t)a.In * K; e += 64) Y[e] = AT(0);
}

// Same, with the row ids known: prev_id = rows[s - 1] (-1 for s = 0), id = rows[s].
template <typename AT>
__device__ inline void zero_gaps_ids(const TtmcArgs& a, int s, int prev_id, int id, int lane) {
    AT* Y = (AT*)a.Y;
    const int64_t K = a.K;
    for (int64_t e = (int64_t)(prev_id + 1) * K + lane; e < (int64_t)id * K; e += 64) Y[e] = AT(0);
    if (s == a.S - 1)
        for (int64_t e = (int64_t)(id + 1) * K + lane; e < (int64_t)a.In * K; e += 64) Y[e] = AT(0);
}

// v + (v of lane l ^ D) for D = 16 or 32, through the lane-swap instructions (no LDS): each lane
// receives both values of its pair, lower lane first, so the two lanes compute the same sum
template <int D>
__device__ inline float pair_sum(float v) {
    const unsigned u = __float_as_uint(v);
    if constexpr (D == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
}

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d4_t __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA tiles: lane l supplies A[l%16][l/16] and B[l/16][l%16]; its 4 results hold
// column l%16 of D, rows 4*(l/16)+v for the fp32 form and l/16+4*v for the fp64 form.
template <typename AT> struct Acc;
template <> struct Acc<float> {
    typedef f4_t type;
    static __device__ inline f4_t mfma(float a, float b, f4_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int kq, int v) { return 4 * kq + v; }
};
template <> struct Acc<double> {
    typedef d4_t type;
    static __device__ inline d4_t mfma(double a, double b, d4_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int kq, int v) { return kq + 4 * v; }
};

template <typename AT> struct Vec4;
template <> struct Vec4<float> { typedef float4 type; };
template <> struct Vec4<double> { typedef double4 type; };

// Order-3 TTMc on MFMA.  A row segment is consumed in batches of 64 nonzeros: the batch's index
// pairs and values are read coalesced (one per lane; the last batch of a segment is padded with
// zero values at a valid index) and staged in the wave's LDS slot.  In a full batch lane group
// g = l/16 takes nonzeros 16g..16g+15 and step s of the 16 MFMAs contracts nonzeros {16g + s}; in
// the last, partial batch step s contracts nonzeros {4s + g} so that ceil(r/4) steps cover r.
// All factor gathers of a batch are issued before its MFMAs, and the next batch's stream loads
// are issued after the gathers (memory counters retire in order, so waiting for the gathers does
// not wait for the prefetch).
template <typename AT, typename ST>
__device__ inline void stage_load(const TtmcArgs& a, const int32_t* __restrict__ ia, const int32_t* __restrict__ ib,
                                  int p, int end, int lane, int& pa, int& pb, AT& px) {
    const int q = p + lane;
    const bool v = q < end;
    const int qc = v ? q : end - 1;
    pa = ia[qc] & kIndexMask;
    pb = ib[qc];
    px = v ? load_as<AT, ST>(a.val, qc) : AT(0);
}

template <typename AT, typename ST>
__global__ __launch_bounds__(256) void k_ttmc3_mfma(TtmcArgs a) {
    __shared__ __align__(32) int32_t s_ia[4][64];
    __shared__ __align__(32) int32_t s_ib[4][64];
    __shared__ __align__(32) AT s_x[4][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int ch = blockIdx.x * 4 + w;
    if (ch >= a.nchunks) return;
    const int kq = lane >> 4;         // lane group: which nonzeros of a step this lane carries
    const int m = lane & 15;          // factor column carried by this lane
    const int q0 = a.chunk_ptr[ch], q1 = a.chunk_ptr[ch + 1];
    const int slot = a.chunk_slot[ch];
    const int32_t* __restrict__ ia = a.idx;
    const int32_t* __restrict__ ib = a.idx + a.nnz;
    // uniform bases with 32-bit per-lane element offsets (global loads with a scalar base)
    const ST* __restrict__ Fa = (const ST*)a.F[0];
    const ST* __restrict__ Fb = (const ST*)a.F[1];
    const int Ra = a.R[0], Rb = a.R[1], K = a.K;
    int s = a.chunk_row[ch];
    int q = q0;
    int pa, pb;
    AT px;
    // first batch of the chunk
    {
        const int end0 = min(a.ptr[s + 1], q1);
        stage_load<AT, ST>(a, ia, ib, q, end0, lane, pa, pb, px);
    }
    while (q < q1) {
        const int rs = a.ptr[s];
        const int end = min(a.ptr[s + 1], q1);
        const bool owner = rs >= q0;
        typename Acc<AT>::type acc = {0, 0, 0, 0};
        for (int p = q; p < end; p += 64) {
            const int r = min(64, end - p);
            s_ia[w][lane] = pa;
            s_ib[w][lane] = pb;
            s_x[w][lane] = px;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // where the next batch starts: this segment, else the next row of the chunk
            const int pn = p + 64 < end ? p + 64 : end;
            const int endn = p + 64 < end ? end : (end < q1 ? min(a.ptr[s + 2], q1) : 0);
            if (r == 64) {
                int ja[16], jb[16];
                AT xs[16];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int4 ta = *(const int4*)&s_ia[w][16 * kq + 4 * v];
                    const int4 tb = *(const int4*)&s_ib[w][16 * kq + 4 * v];
                    const typename Vec4<AT>::type tx = *(const typename Vec4<AT>::type*)&s_x[w][16 * kq + 4 * v];
                    ja[4 * v] = ta.x; ja[4 * v + 1] = ta.y; ja[4 * v + 2] = ta.z; ja[4 * v + 3] = ta.w;
                    jb[4 * v] = tb.x; jb[4 * v + 1] = tb.y; jb[4 * v + 2] = tb.z; jb[4 * v + 3] = tb.w;
                    xs[4 * v] = tx.x; xs[4 * v + 1] = tx.y; xs[4 * v + 2] = tx.z; xs[4 * v + 3] = tx.w;
                }
                AT av[16], bv[16];
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    av[t] = load_as<AT, ST>(Fa, (uint32_t)(ja[t] * 16 + m));
                    bv[t] = load_as<AT, ST>(Fb, (uint32_t)(jb[t] * 16 + m));
                }
                __builtin_amdgcn_sched_barrier(0);
                if (pn < endn) stage_load<AT, ST>(a, ia, ib, pn, endn, lane, pa, pb, px);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int t = 0; t < 16; ++t) acc = Acc<AT>::mfma(av[t] * xs[t], bv[t], acc);
            } else {
                const int ngroups = (r + 15) >> 4;   // groups of 4 steps of 4 nonzeros
                AT av[16], bv[16];
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    if ((t >> 2) < ngroups) {
                        const int e = 4 * t + kq;
                        av[t] = load_as<AT, ST>(Fa, (uint32_t)(s_ia[w][e] * 16 + m)) * s_x[w][e];
                        bv[t] = load_as<AT, ST>(Fb, (uint32_t)(s_ib[w][e] * 16 + m));
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                if (pn < endn) stage_load<AT, ST>(a, ia, ib, pn, endn, lane, pa, pb, px);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int t = 0; t < 16; ++t)
                    if ((t >> 2) < ngroups) acc = Acc<AT>::mfma(av[t], bv[t], acc);
            }
        }
        AT* dst = owner ? (AT*)a.Y + (int64_t)a.rows[s] * K : (AT*)a.carry + (int64_t)slot * K;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = Acc<AT>::row(kq, v);
            if (rr < Ra && m < Rb) dst[rr * Rb + m] = acc[v];
        }
        if (owner) zero_gaps<AT>(a, s, lane);
        q = end;
        ++s;
    }
}

// Order-3 TTMc (R_a, R_b <= 16) on FP32 MFMA (the library runs it on FP32 storage; BF16 storage
// takes k_ttmc3_bf below, whose batch pipeline is the same), walking the padded stream
// of a chunk in batches of 64 entries regardless of row boundaries (rows are padded to whole
// 4-entry steps).  Software pipeline per wave, iteration b:
//   1. read batch b's factor rows (from the wave's LDS tile) and values into registers;
//   2. stage batch b+1's index pairs and values (loaded two iterations earlier) in LDS and gather
//      its 64 + 64 factor rows into registers with 16-byte loads (4 lanes per FP32 row of 64 B,
//      2 per BF16 row of 32 B), then issue the stream loads of batch b+3;
//   3. run batch b's 16 MFMA steps - the gathers are in flight meanwhile;
//   4. write batch b+1's rows into the LDS tile (waiting only for the gathers: memory counters
//      retire in order and the later stream loads may stay in flight).
// Step t contracts entries 4t..4t+3 (lane l carries entry 4t + l/16 and factor column l%16) with
// v_mfma_f32_16x16x4f32; a step whose first entry carries the row flag first writes out the
// finished row.
template <typename ST>
struct LdsTiles {
    ST A[64 * 16];
    ST B[64 * 16];
    float x[2][64];      // entry n at (n % 4) * 16 + n / 4
    int32_t ia[64];
    int32_t ib[64];
};

// Residual form (the adjoint of the completion loss): the value of each entry is replaced by its
// residual e = xhat - x, computed from the rows already in the tile.  With M = row i_n of
// U_n G_(n) as an R_a x R_b matrix, xhat = a^T M b; a tile of 16 entries of one row takes four
// 16x16x4 MFMAs for M [b_1 .. b_16] (lane l supplies M[l%16][4(l/16)+c] and b_{l%16}[4(l/16)+c]
// in MFMA c, so one 16-byte LDS read of the B row and one 16-byte load of M serve all four), and
// lane l then holds rows 4(l/16)..+3 of column l%16: a 4-term dot with the matching part of a
// and two cross-lane additions give xhat.  A tile that spans several rows repeats the MFMAs per
// row.  M of the first two rows of the next batch is loaded one batch ahead (other rows, which
// occur only for rows shorter than a batch, are loaded on demand).  Padding entries repeat the
// indices of their row's last entry and coordinates are distinct after coalescing, so an entry
// that opens no row and repeats its predecessor's indices is padding: its residual is 0.
// s_waitcnt immediate for vmcnt(0) with the other counters left free (expcnt 7, lgkmcnt 15)
constexpr int kWaitVm0 = 0x0F70;

struct ResArgs {
    const float* W;      // [I_n][16 x 16]: row i_n of U_n G_(n), entry (r_a, r_b) at 16 r_a + r_b
    double* part;        // per-chunk sum of squared residuals, or null
};

template <typename ST, bool RES>
__global__ __launch_bounds__(256) void k_ttmc3_lds(TtmcArgs a, ResArgs res) {
    static_assert(!RES || sizeof(ST) == 4, "the residual form reads FP32 tiles");
    constexpr int ROWB = 16 * (int)sizeof(ST);   // bytes of one padded factor row
    constexpr int LPR = ROWB / 16;               // lanes per row in a 16-byte gather
    constexpr int RPI = 64 / LPR;                // rows per gather instruction
    constexpr int NI = 64 / RPI;                 // gather instructions per factor per batch
    __shared__ __align__(16) LdsTiles<ST> tiles[4];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int ch = blockIdx.x * 4 + w;
    if (ch >= a.nchunks) return;
    LdsTiles<ST>& T = tiles[w];
    const int kq = lane >> 4, m = lane & 15;
    const int q0 = a.chunk_ptr[ch], q1 = a.chunk_ptr[ch + 1];
    const int slot = a.chunk_slot[ch];
    const int32_t* __restrict__ ia = a.idx;
    const int32_t* __restrict__ ib = a.idx + a.nnz;
    const char* __restrict__ Fa = (const char*)a.F[0];
    const char* __restrict__ Fb = (const char*)a.F[1];
    const int Ra = a.R[0], Rb = a.R[1], K = a.K;
    const int s0 = a.chunk_row[ch];
    int s = s0;
    f4_t acc = {0, 0, 0, 0};

    // the chunk owns every row it holds except a first row that started in an earlier chunk
    // row ids of the rows a batch may touch, rows[rbase + lane] (a batch holds at most 16 rows),
    // loaded one batch ahead; prev_id = id of the row before the one being finished
    int rbase = s0;
    int rowsv = ld_const(a.rows, min(s0 + lane, a.S - 1));
    int prev_id = (s0 > 0) ? ld_const(a.rows, s0 - 1) : -1;
    auto flush = [&](int row) __attribute__((always_inline)) {
        const bool owner = (row != s0) || (slot < 0);
        const int id = __builtin_amdgcn_readlane(rowsv, row - rbase);
        const uint64_t base = owner ? (uint64_t)(uintptr_t)a.Y : (uint64_t)(uintptr_t)a.carry;
        const int64_t off = owner ? (int64_t)id * K : (int64_t)slot * K;
        float* dst = (float*)(uintptr_t)base + off;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 4 * kq + v;
            if (r < Ra && m < Rb) dst[r * Rb + m] = acc[v];
        }
        if (owner && (id != prev_id + 1 || row == a.S - 1)) zero_gaps_ids<float>(a, row, prev_id, id, lane);
        prev_id = id;
    };
    auto stream_load = [&](int pstart, int& ra, int& rb, float& rx) __attribute__((always_inline)) {
        const int qq = pstart + lane;
        const bool v = qq < q1;
        if constexpr (RES) {
            // unconditional loads at a clamped position: with no branch around them the compiler
            // counts them exactly, and later waits leave the gathers in flight
            const int qc = max(min(qq, q1 - 1), 0);
            const int ta = ia[qc], tb = ib[qc];
            const float tx = load_as<float, ST>(a.val, qc);
            ra = v ? ta : 0;
            rb = v ? tb : 0;
            rx = v ? tx : 0.f;
        } else {
            ra = v ? ia[qq] : 0;
            rb = v ? ib[qq] : 0;
            rx = v ? load_as<float, ST>(a.val, qq) : 0.f;
        }
    };
    // residual form: indices of the entry before the batch, and the padding mask of a batch
    int last_a = -1, last_b = -1;
    if constexpr (RES) {
        if (q0 > 0) {
            last_a = ia[q0 - 1] & kIndexMask;
            last_b = ib[q0 - 1];
        }
    }
    // stage a batch starting at pstart; in the residual form keep = this lane's entry is a real
    // one (not padding, not past the chunk end), and the values go to the tile only as residuals
    auto stage = [&](int xb, int ra, int rb, float rx, int pstart, bool& keep) __attribute__((always_inline)) -> uint64_t {
        const uint64_t st = __ballot(ra < 0);
        if constexpr (RES) {
            const int ma = ra & kIndexMask;
            int pa = __shfl(ma, (lane + 63) & 63);
            int pb = __shfl(rb, (lane + 63) & 63);
            if (lane == 0) {
                pa = last_a;
                pb = last_b;
            }
            keep = pstart + lane < q1 && !(ra >= 0 && ma == pa && rb == pb);
            last_a = __builtin_amdgcn_readlane(ma, 63);
            last_b = __builtin_amdgcn_readlane(rb, 63);
        }
        T.ia[lane] = ra & kIndexMask;
        T.ib[lane] = rb;
        if constexpr (!RES) T.x[xb][(lane & 3) * 16 + (lane >> 2)] = rx;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        return st;
    };
    // gathered rows of one batch, in named registers (16 bytes of a factor-A and a factor-B row
    // per lane and instruction; NI <= 4)
    static_assert(NI <= 4, "gather registers");
#define TK_G1(j, va, vb)                                                                            \
    if constexpr (NI > j) {                                                                         \
        const int row = j * RPI + lane / LPR;                                                       \
        const uint32_t part = (uint32_t)(lane % LPR) * 16u;                                         \
        va = *(const uint4*)(Fa + ((uint32_t)T.ia[row] * (uint32_t)ROWB + part));                   \
        vb = *(const uint4*)(Fb + ((uint32_t)T.ib[row] * (uint32_t)ROWB + part));                   \
    }
#define TK_P1(j, va, vb)                                                                            \
    if constexpr (NI > j) {                                                                         \
        *(uint4*)((char*)T.A + j * 1024 + put_off) = va;                                            \
        *(uint4*)((char*)T.B + j * 1024 + put_off) = vb;                                            \
    }
#define TK_GATHER()                                                                                 \
    TK_G1(0, ga0, gb0) TK_G1(1, ga1, gb1) TK_G1(2, ga2, gb2) TK_G1(3, ga3, gb3)
#define TK_PUT()                                                                                    \
    TK_P1(0, ga0, gb0) TK_P1(1, ga1, gb1) TK_P1(2, ga2, gb2) TK_P1(3, ga3, gb3)                     \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");                                          \
    __builtin_amdgcn_wave_barrier();                                                                \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint4 ga0, ga1, ga2, ga3, gb0, gb1, gb2, gb3;
    // Tile layout.  The residual form reads 16-byte column groups of 16 different entries at a
    // row stride of 64 bytes, which would fall on the same banks: there the group g of entry n is
    // stored at group g ^ ((n >> 2) & 3) (a permutation within the row, so the column reads of the
    // MFMA steps stay conflict-free too: column c of entry e sits at c ^ (4 ((e >> 2) & 3))).
    // The gather puts lane l's 16 bytes (entry 16 j + l / 4, group l % 4) into the tile.
    const int put_off = RES ? (lane >> 2) * 64 + 16 * ((lane & 3) ^ ((lane >> 4) & 3)) : lane * 16;

    // residual form: M of rows mr0 and mr1 (16 bytes of each per lane), the wave's sum of e^2
    float4 Mc0 = make_float4(0.f, 0.f, 0.f, 0.f), Mc1 = Mc0;
    int mr0 = -1, mr1 = -1;
    double e2sum = 0.0;
    const float* const Wlane = res.W + m * 16 + 4 * kq;   // this lane's 16 bytes of a block
    auto loadM = [Wlane](int id) __attribute__((always_inline)) -> float4 { return *(const float4*)(Wlane + (int64_t)id * 256); };
    // the first two rows of a batch whose first row index is sfirst and row flags are opens
    auto fetch_pair = [&](int sfirst, uint64_t opens, int rows_lane) __attribute__((always_inline)) {
        const int nr0 = sfirst + (int)(opens & 1ull);
        if (nr0 != mr0) {
            if (nr0 == mr1) Mc0 = Mc1;
            else Mc0 = loadM(__builtin_amdgcn_readlane(rows_lane, nr0 - sfirst));
            mr0 = nr0;
        }
        if ((opens & ~1ull) != 0 && mr1 != nr0 + 1) {
            Mc1 = loadM(__builtin_amdgcn_readlane(rows_lane, nr0 + 1 - sfirst));
            mr1 = nr0 + 1;
        }
    };

    // prologue: batch 0 staged and its rows in LDS; stream registers for batches 1 and 2
    int r1a = 0, r1b = 0, r2a = 0, r2b = 0;
    float r1x = 0.f, r2x = 0.f;
    uint64_t starts;
    bool keep = false;     // residual form: this lane's entry of the current batch is real
    float xcur = 0.f;      // residual form: its value
    {
        int r0a, r0b;
        float r0x;
        stream_load(q0, r0a, r0b, r0x);
        if (q0 + 64 < q1) stream_load(q0 + 64, r1a, r1b, r1x);
        if (q0 + 128 < q1) stream_load(q0 + 128, r2a, r2b, r2x);
        starts = stage(0, r0a, r0b, r0x, q0, keep);
        xcur = r0x;
        if constexpr (RES) fetch_pair(s0, starts & ~1ull, rowsv);
        TK_GATHER()
        TK_PUT()
    }
    int xb = 0;
    for (int p = q0; p < q1; p += 64) {
        const int nsteps = min(16, (q1 - p) >> 2);
        const bool plain = starts == 0 || (starts == 1ull && p == q0);   // no row opens inside
        // 1. stage batch b+1 (past the chunk end: zero values at row 0), gather its rows, then the
        //    stream loads of batch b+3; the gathers fly while batch b runs
        bool keep_next = false;
        const float xnext = r1x;
        const uint64_t starts_next = stage(xb ^ 1, r1a, r1b, r1x, p + 64, keep_next);
        // first row of batch b+1: this batch's row plus the rows opened inside it
        const int s_next = s + __popcll(starts & ~((p == q0) ? 1ull : 0ull));
        const int rows_next = ld_const(a.rows, min(s_next + lane, a.S - 1));
        TK_GATHER()
        r1a = r2a; r1b = r2b; r1x = r2x;
        if (RES || p + 192 < q1) stream_load(p + 192, r2a, r2b, r2x);
        if constexpr (RES) {
            // residuals of batch b into its value slots (padding and entries past the end: 0)
            const int nvalid = min(64, q1 - p);
            const uint64_t opens = starts & ~((p == q0) ? 1ull : 0ull);
            auto upto = [](int n) __attribute__((always_inline)) -> uint64_t { return (n >= 63) ? ~0ull : ((2ull << n) - 1); };
            // M of row rr: slot 0 or 1; a third row in one batch is loaded into slot 1 and waited
            // for there, so that the common path keeps the gathers in flight
#define TK_PICK_M(rr, M)                                                                            \
    if ((rr) != mr0 && (rr) != mr1) {                                                               \
        Mc1 = loadM(__builtin_amdgcn_readlane(rowsv, (rr) - s));                                    \
        mr1 = (rr);                                                                                 \
        __builtin_amdgcn_s_waitcnt(kWaitVm0);                                                       \
    }                                                                                               \
    float4 M = Mc1;                                                                                 \
    if ((rr) == mr0) M = Mc0;
            auto tile_model = [](float4 M, float4 bq, float4 aq) __attribute__((always_inline)) -> float {
                f4_t d = {0, 0, 0, 0};
                d = Acc<float>::mfma(M.x, bq.x, d);
                d = Acc<float>::mfma(M.y, bq.y, d);
                d = Acc<float>::mfma(M.z, bq.z, d);
                d = Acc<float>::mfma(M.w, bq.w, d);
                return ((d[0] * aq.x + d[1] * aq.y) + d[2] * aq.z) + d[3] * aq.w;
            };
            float mine = 0.f;   // model value of entry `lane` of the batch
#pragma unroll 1
            for (int j = 0; j < 4; ++j) {
                if (16 * j < nvalid) {
                    const int n = 16 * j + m;
                    const int col = n * 16 + 4 * (kq ^ ((m >> 2) & 3));   // group kq of entry n
                    const float4 bq = *(const float4*)((const float*)T.B + col);
                    const float4 aq = *(const float4*)((const float*)T.A + col);
                    // rows of the tile: the row of entry 16 j and one more per row opened inside
                    const int rlo = s + __popcll(opens & upto(16 * j));
                    const int rhi = rlo + __popcll(opens & (0xFFFEull << (16 * j)));
                    float xh;
                    if (rlo == rhi) {
                        TK_PICK_M(rlo, M0)
                        xh = tile_model(M0, bq, aq);
                    } else {
                        const int rme = s + __popcll(opens & upto(n));
                        xh = 0.f;
                        for (int rr = rlo; rr <= rhi; ++rr) {
                            TK_PICK_M(rr, Mr)
                            const float part = tile_model(Mr, bq, aq);
                            if (rr == rme) xh = part;
                        }
                    }
#undef TK_PICK_M
                    xh = pair_sum<16>(xh);
                    xh = pair_sum<32>(xh);
                    if (kq == j) mine = xh;
                }
            }
            const float e = keep ? mine - xcur : 0.f;
            T.x[xb][(lane & 3) * 16 + (lane >> 2)] = e;
            e2sum += (double)e * (double)e;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // M of batch b+1's first two rows: issued after the gathers, so the tile writes at
            // the end of the iteration do not wait for them
            fetch_pair(s_next, starts_next, rows_next);
        }
        // 2. batch b's MFMA steps from the LDS tile
        auto operand = [&](int t, float& av, float& bv) __attribute__((always_inline)) {
            const int e = (4 * t + kq) * 16 + (RES ? (m ^ (4 * (t & 3))) : m);
            if constexpr (sizeof(ST) == 4) { av = T.A[e]; bv = T.B[e]; }
            else { av = bf16_to_f32(T.A[e]); bv = bf16_to_f32(T.B[e]); }
            av *= T.x[xb][kq * 16 + t];
        };
        // (the residual form, which holds more registers, reads the operands in two halves)
        constexpr int CH = RES ? 4 : 16;
        if (plain) {
#pragma unroll
            for (int t0 = 0; t0 < 16; t0 += CH) {
                float av[CH], bv[CH];
#pragma unroll
                for (int t = 0; t < CH; ++t) operand(t0 + t, av[t], bv[t]);
#pragma unroll
                for (int t = 0; t < CH; ++t)
                    if (t0 + t < nsteps) acc = Acc<float>::mfma(av[t], bv[t], acc);
            }
        } else {
            // rows open inside the batch: the operands are read first, then the unrolled steps
            // write a finished row out before the step that opens the next one
            const uint64_t opens = starts & ~((p == q0) ? 1ull : 0ull);
#pragma unroll
            for (int t0 = 0; t0 < 16; t0 += CH) {
                float av[CH], bv[CH];
#pragma unroll
                for (int t = 0; t < CH; ++t) operand(t0 + t, av[t], bv[t]);
#pragma unroll
                for (int t = 0; t < CH; ++t) {
                    if (t0 + t < nsteps) {
                        if ((opens >> (4 * (t0 + t))) & 1ull) {
                            flush(s);
                            ++s;
                            acc = f4_t{0, 0, 0, 0};
                        }
                        acc = Acc<float>::mfma(av[t], bv[t], acc);
                    }
                }
            }
        }
        // 4. batch b+1's rows into the tile
        TK_PUT()
        starts = starts_next;
        keep = keep_next;
        xcur = xnext;
        xb ^= 1;
        rbase = s_next;
        rowsv = rows_next;
    }
    flush(s);
    if constexpr (RES) {
        if (res.part) {
            for (int o = 32; o > 0; o >>= 1) e2sum += __shfl_xor(e2sum, o);
            if (lane == 0) res.part[ch] = e2sum;
        }
    }
#undef TK_G1
#undef TK_P1
#undef TK_GATHER
#undef TK_PUT
}

// Order-3 TTMc with BF16 operands on the BF16 matrix instruction (v_mfma_f32_16x16x32_bf16, 32
// nonzeros per instruction).  That instruction takes, in lane l, eight consecutive values of the
// contraction index (nonzeros 8(l/16)..+7) for one factor column l%16, while a 16-byte gather holds
// eight columns of one nonzero's row: the wave's tile stays entry-major (as gathered, with the A
// row scaled: A[e] = bf16(x_e a_e), the product of two BF16 numbers exact in FP32 and rounded once
// to BF16 as it is written) and the operands are read column-wise, 2 bytes per value.  The 32-byte
// rows sit four to a 128-byte group with row e in slot (e & 3) ^ ((e >> 3) & 3), so that both the
// 16-byte row writes and the column reads of 4 x 16 (entry, column) pairs fall on distinct banks.
// The batch pipeline is that of the FP32-tile kernel above (stream two batches ahead, rows
// gathered one batch ahead with 16-byte loads, two lanes per 32-byte row).  A batch that lies
// inside one row takes two MFMAs; a batch in which rows open takes the 16 FP32 steps of four
// nonzeros each (v_mfma_f32_16x16x4f32 on the same tile values), writing each finished row out
// before the step that opens the next.  Either way every product is bf16(x a) * b, exact in FP32,
// and the sums are FP32.
struct BfTiles {
    uint4 A[128];   // 64 rows of 16 BF16 values, swizzled (bf_off)
    uint4 B[128];
    float x[64];
    int32_t ia[64];
    int32_t ib[64];
};

// byte offset of column c of entry e in a tile
__device__ inline uint32_t bf_off(int e, int c) {
    return 128u * (uint32_t)(e >> 2) + 32u * (uint32_t)((e & 3) ^ ((e >> 3) & 3)) + 2u * (uint32_t)c;
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_ttmc3_bf(TtmcArgs a) {
    constexpr int ROWB = 32;   // bytes of one padded BF16 factor row
    __shared__ __align__(16) BfTiles tiles[4];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int ch = blockIdx.x * 4 + w;
    if (ch >= a.nchunks) return;
    BfTiles& T = tiles[w];
    const int kq = lane >> 4, m = lane & 15;
    const int q0 = a.chunk_ptr[ch], q1 = a.chunk_ptr[ch + 1];
    const int slot = a.chunk_slot[ch];
    const int32_t* __restrict__ ia = a.idx;
    const int32_t* __restrict__ ib = a.idx + a.nnz;
    const char* __restrict__ Fa = (const char*)a.F[0];
    const char* __restrict__ Fb = (const char*)a.F[1];
    const int Ra = a.R[0], Rb = a.R[1], K = a.K;
    const int s0 = a.chunk_row[ch];
    int s = s0;
    f4_t acc = {0, 0, 0, 0};

    // rows of the chunk: as in the FP32-tile kernel
    int rbase = s0;
    int rowsv = ld_const(a.rows, min(s0 + lane, a.S - 1));
    int prev_id = (s0 > 0) ? ld_const(a.rows, s0 - 1) : -1;
    auto flush = [&](int row) __attribute__((always_inline)) {
        const bool owner = (row != s0) || (slot < 0);
        const int id = __builtin_amdgcn_readlane(rowsv, row - rbase);
        const uint64_t base = owner ? (uint64_t)(uintptr_t)a.Y : (uint64_t)(uintptr_t)a.carry;
        const int64_t off = owner ? (int64_t)id * K : (int64_t)slot * K;
        float* dst = (float*)(uintptr_t)base + off;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 4 * kq + v;
            if (r < Ra && m < Rb) dst[r * Rb + m] = acc[v];
        }
        if (owner && (id != prev_id + 1 || row == a.S - 1)) zero_gaps_ids<float>(a, row, prev_id, id, lane);
        prev_id = id;
    };
    // stream loads at a clamped position, with no branch around them and the raw BF16 value kept:
    // entries past the chunk end are masked (index 0, value 0) only when the batch is staged, so
    // no wait for the stream holds up the gathers in flight
    auto stream_load = [&](int pstart, int& ra, int& rb, int& rx) __attribute__((always_inline)) {
        const int qc = max(min(pstart + lane, q1 - 1), 0);
        ra = ia[qc];
        rb = ib[qc];
        rx = ((const bf16_t*)a.val)[qc];
    };
    auto stage = [&](int ra, int rb, int rx, int pstart) __attribute__((always_inline)) -> uint64_t {
        const bool v = pstart + lane < q1;
        ra = v ? ra : 0;
        rb = v ? rb : 0;
        const uint64_t st = __ballot(ra < 0);
        T.ia[lane] = ra & kIndexMask;
        T.ib[lane] = rb;
        T.x[lane] = v ? bf16_to_f32((bf16_t)rx) : 0.f;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        return st;
    };
    // gather instruction j: lane l loads 16 bytes (columns 8(l%2)..+7) of entry 32 j + l/2
    uint4 ga0, ga1, gb0, gb1;
    auto gather = [&]() __attribute__((always_inline)) {
        const uint32_t part = (uint32_t)(lane & 1) * 16u;
        const int r0 = lane >> 1, r1 = 32 + (lane >> 1);
        ga0 = *(const uint4*)(Fa + ((uint32_t)T.ia[r0] * (uint32_t)ROWB + part));
        gb0 = *(const uint4*)(Fb + ((uint32_t)T.ib[r0] * (uint32_t)ROWB + part));
        ga1 = *(const uint4*)(Fa + ((uint32_t)T.ia[r1] * (uint32_t)ROWB + part));
        gb1 = *(const uint4*)(Fb + ((uint32_t)T.ib[r1] * (uint32_t)ROWB + part));
    };
    // the gathered rows into the tile (16 bytes per lane and factor), a scaled by the entry's value
    auto put_one = [&](const uint4& ua, const uint4& ub, int e) __attribute__((always_inline)) {
        const float xe = T.x[e];
        const uint32_t wa[4] = {ua.x, ua.y, ua.z, ua.w};
        uint32_t pa[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float lo = __uint_as_float(wa[i] << 16) * xe;
            const float hi = __uint_as_float(wa[i] & 0xffff0000u) * xe;
            const bf16x2_t p = __builtin_convertvector((float __attribute__((ext_vector_type(2)))){lo, hi}, bf16x2_t);
            pa[i] = __builtin_bit_cast(uint32_t, p);
        }
        const uint32_t off = bf_off(e, 8 * (lane & 1));
        *(uint4*)((char*)T.A + off) = make_uint4(pa[0], pa[1], pa[2], pa[3]);
        *(uint4*)((char*)T.B + off) = ub;
    };
    auto put = [&]() __attribute__((always_inline)) {
        put_one(ga0, gb0, lane >> 1);
        put_one(ga1, gb1, 32 + (lane >> 1));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };

    // prologue: batch 0 staged and its rows in the tile; stream registers for batches 1 and 2
    int r1a, r1b, r2a, r2b, r1x, r2x;
    uint64_t starts;
    {
        int r0a, r0b, r0x;
        stream_load(q0, r0a, r0b, r0x);
        stream_load(q0 + 64, r1a, r1b, r1x);
        stream_load(q0 + 128, r2a, r2b, r2x);
        starts = stage(r0a, r0b, r0x, q0);
        gather();
        put();
    }
    // one batch: ra/rb/rx hold batch b+1 and then receive batch b+3 (the loop below alternates two
    // register sets, so that no copy waits for a stream load in flight)
    auto batch = [&](int p, int& ra, int& rb, int& rx) __attribute__((always_inline)) {
        const int nsteps = min(16, (q1 - p) >> 2);
        const bool plain = starts == 0 || (starts == 1ull && p == q0);   // no row opens inside
        // 1. stage batch b+1, gather its rows, then the stream loads of batch b+3
        const uint64_t starts_next = stage(ra, rb, rx, p + 64);
        const int s_next = s + __popcll(starts & ~((p == q0) ? 1ull : 0ull));
        const int rows_next = ld_const(a.rows, min(s_next + lane, a.S - 1));
        gather();
        stream_load(p + 192, ra, rb, rx);
        // 2. batch b from the tile
        if (plain) {
            // entries past the chunk end carry zero values
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (32 * j < q1 - p) {
                    bf16x8_t av, bv;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const uint32_t off = bf_off(32 * j + 8 * kq + i, m);
                        av[i] = *(const __bf16*)((const char*)T.A + off);
                        bv[i] = *(const __bf16*)((const char*)T.B + off);
                    }
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
                }
            }
        } else {
            // rows open inside the batch: step t contracts entries 4t..4t+3 (lane l: entry
            // 4t + l/16, column l%16); a finished row is written before the step opening the next
            const uint64_t opens = starts & ~((p == q0) ? 1ull : 0ull);
#pragma unroll
            for (int t0 = 0; t0 < 16; t0 += 8) {
                float av[8], bv[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const uint32_t off = bf_off(4 * (t0 + t) + kq, m);
                    av[t] = bf16_to_f32(*(const bf16_t*)((const char*)T.A + off));
                    bv[t] = bf16_to_f32(*(const bf16_t*)((const char*)T.B + off));
                }
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    if (t0 + t < nsteps) {
                        if ((opens >> (4 * (t0 + t))) & 1ull) {
                            flush(s);
                            ++s;
                            acc = f4_t{0, 0, 0, 0};
                        }
                        acc = Acc<float>::mfma(av[t], bv[t], acc);
                    }
                }
            }
        }
        // 3. batch b+1's rows into the tile
        put();
        starts = starts_next;
        rbase = s_next;
        rowsv = rows_next;
    };
    for (int p = q0; p < q1; p += 128) {
        batch(p, r1a, r1b, r1x);
        if (p + 64 >= q1) break;
        batch(p + 64, r2a, r2b, r2x);
    }
    flush(s);
}

template <typename AT, typename ST, int KPL>
__global__ __launch_bounds__(256) void k_ttmc_generic(TtmcArgs a) {
    extern __shared__ uint16_t dig[];  // [K][nm1]: digit of each other mode for column c
    for (int c = threadIdx.x; c < a.K; c += blockDim.x) {
        int rem = c;
        for (int j = a.nm1 - 1; j >= 0; --j) {
            dig[c * a.nm1 + j] = (uint16_t)(rem % a.R[j]);
            rem /= a.R[j];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int ch = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    if (ch >= a.nchunks) return;
    const int q0 = a.chunk_ptr[ch], q1 = a.chunk_ptr[ch + 1];
    const int slot = a.chunk_slot[ch];
    const int K = a.K, nm1 = a.nm1;
    int s = a.chunk_row[ch];
    int q = q0;
    while (q < q1) {
        const int rs = a.ptr[s];
        const int end = min(a.ptr[s + 1], q1);
        const bool owner = rs >= q0;
        AT acc[KPL];
#pragma unroll
        for (int j = 0; j < KPL; ++j) acc[j] = AT(0);
        // unrolled so that the loads of several nonzeros are in flight together
#pragma unroll 4
        for (int p = q; p < end; ++p) {
            const AT x = load_as<AT, ST>(a.val, p);
            int64_t base[kMaxOrder - 1];
#pragma unroll
            for (int t = 0; t < kMaxOrder - 1; ++t)
                base[t] = (t < nm1) ? (int64_t)(a.idx[(int64_t)t * a.nnz + p] & kIndexMask) * a.ld[t] : 0;
#pragma unroll
            for (int j = 0; j < KPL; ++j) {
                const int c = lane + 64 * j;
                if (c < K) {
                    AT v = x;
#pragma unroll
                    for (int t = 0; t < kMaxOrder - 1; ++t)
                        if (t < nm1) v *= load_as<AT, ST>(a.F[t], base[t] + dig[c * nm1 + t]);
                    acc[j] += v;
                }
            }
        }
        AT* dst = owner ? (AT*)a.Y + (int64_t)a.rows[s] * K : (AT*)a.carry + (int64_t)slot * K;
#pragma unroll
        for (int j = 0; j < KPL; ++j) {
            const int c = lane + 64 * j;
            if (c < K) dst[c] = acc[j];
        }
        if (owner) zero_gaps<AT>(a, s, lane);
        q = end;
        ++s;
    }
}

// Order >= 4, fiber-factored (the Kronecker row of a nonzero is (kron of its inner modes' rows)
// kron U_f(i_f, :), f the last other mode).  Within a row the nonzeros are sorted by i_f, so the
// nonzeros sharing i_f form a fiber, and
//     Y_(n)(i_n, :) = sum_fibers  s_fiber kron U_f(i_f, :),   s_fiber = sum_p x_p kron_inner(p),
// which needs Ks = prod_inner R products per nonzero and Ks * R_f per fiber instead of K_n per
// nonzero.  Lane l owns the inner columns cs = l + 64 j (j < KSL) and keeps s and the row
// accumulator Y[cs][0..R_f) in registers.
// Per batch of 64 nonzeros (one per lane) the wave stages the inner factor rows transposed
// (column-major: value c of nonzero e at c * kFiberStride + e) and the fiber rows in its LDS slot;
// the index loads run two batches ahead and the 16-byte row loads one batch ahead, so both are in
// flight while the previous batch is walked.  The walk takes four nonzeros at a time: one 16-byte
// LDS read per inner mode gives a lane its factor values of all four.  A nonzero that starts a
// fiber first folds the finished fiber into the row (R_f FMAs per column) and loads the new fiber
// row; a nonzero that starts a row writes the finished row.  Summation order is fixed: the result
// is deterministic.
struct FiberArgs {
    int32_t nin;                   // inner modes (other modes but the fiber mode)
    int32_t off[kMaxOrder - 2];    // offset of inner mode k's row in a staged tile row
    int32_t Rin[kMaxOrder - 2];
    int32_t Rf;
    int32_t Ks;                    // prod_inner R
    int32_t tw;                    // staged values per nonzero: sum_inner R (<= kFiberTile)
    // optional: the inner sum of every fiber piece (a fiber, or its part inside one chunk) is
    // also written to memo[piece][Ks], pieces numbered in stream order from pid_base[chunk]
    void* memo;
    const int32_t* pid_base;
};

constexpr int kFiberTile = 32;

constexpr int kFiberStride = 68;   // transposed tile row: 64 nonzeros + 4 (16-byte aligned rows)

template <typename AT, int RF>
__host__ __device__ constexpr int fiber_slot_words(int tw) {
    // in[tw][kFiberStride] (transposed), uf[64][RF], x[64]  (in units of AT)
    return tw * kFiberStride + 64 * RF + 64;
}

template <typename AT, typename ST, int NM1, int KSL, int RF, int LDC>
__global__ __launch_bounds__(256) void k_ttmc_fiber(TtmcArgs a, FiberArgs f) {
    extern __shared__ __align__(16) unsigned char fiber_lds[];
    constexpr int NV = LDC * (int)sizeof(ST) / 16;  // 16-byte loads per factor row (LDC columns)
    static_assert(RF <= LDC || LDC == 16, "fiber rows narrower than the staged tile");
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ch = blockIdx.x * 4 + w;
    if (ch >= a.nchunks) return;
    typedef AT at4 __attribute__((ext_vector_type(4)));
    AT* Tin = (AT*)fiber_lds + (size_t)w * fiber_slot_words<AT, RF>(f.tw);
    AT* Tuf = Tin + f.tw * kFiberStride;
    AT* Tx = Tuf + 64 * RF;
    const int q0 = a.chunk_ptr[ch], q1 = a.chunk_ptr[ch + 1];
    const int slot = a.chunk_slot[ch];
    const int s0 = a.chunk_row[ch];
    const int K = a.K, Rf = f.Rf;
    // tile offsets of this lane's inner columns (loops unrolled: the arrays stay in registers)
    int toff[KSL][NM1 - 1];
#pragma unroll
    for (int j = 0; j < KSL; ++j) {
        int rem = lane + 64 * j;
#pragma unroll
        for (int k = NM1 - 2; k >= 0; --k) {
            toff[j][k] = f.off[k] + rem % f.Rin[k];
            rem /= f.Rin[k];
        }
    }
    AT sacc[KSL], yacc[KSL][RF], u[RF];
#pragma unroll
    for (int j = 0; j < KSL; ++j) {
        sacc[j] = AT(0);
#pragma unroll
        for (int r = 0; r < RF; ++r) yacc[j][r] = AT(0);
    }
#pragma unroll
    for (int r = 0; r < RF; ++r) u[r] = AT(0);
    int srow = s0;
    int prev_if = -1;

    // prefetch registers: indices and value of the next-but-one batch, rows of the next batch
    // (indices in a 4-vector, NM1 <= 4, so they stay in registers)
    typedef int32_t i4v __attribute__((ext_vector_type(4)));
    static_assert(NM1 <= 4, "fiber kernel: order <= 5");
    i4v i1 = {0, 0, 0, 0}, i2 = {0, 0, 0, 0};
    AT x1 = AT(0), x2 = AT(0);
    uint4 raw[NM1][NV];
    auto load_idx = [&](int p, i4v& ix, AT& xv) __attribute__((always_inline)) {
        const int qq = p + lane;
        const bool v = qq < q1;
        const int qc = v ? qq : q1 - 1;
#pragma unroll
        for (int t = 0; t < NM1; ++t) ix[t] = a.idx[(int64_t)t * a.nnz + qc];
        xv = load_as<AT, ST>(a.val, (int64_t)qc);
    };
    // the fiber-mode row is read only by a nonzero that starts a fiber (the walk reads it there
    // alone); last_f: fiber index of the previous batch's last nonzero (-1 at the chunk start)
    int last_f = -1;
    auto load_rows = [&](const i4v ix) __attribute__((always_inline)) {
        int prevf = __shfl_up(ix[NM1 - 1], 1);
        if (lane == 0) prevf = last_f;
        last_f = __builtin_amdgcn_readlane(ix[NM1 - 1], 63);
        const bool fst = ix[0] < 0 || ix[NM1 - 1] != prevf;
#pragma unroll
        for (int t = 0; t < NM1; ++t) {
            const int32_t it = (t == 0) ? (ix[0] & kIndexMask) : ix[t];
            const uint4* row = (const uint4*)((const ST*)a.F[t] + (int64_t)it * a.ld[t]);
            if (t < NM1 - 1 || fst) {
#pragma unroll
                for (int v = 0; v < NV; ++v) raw[t][v] = row[v];
            }
        }
    };
    // fiber sums: this lane's place in the next piece's row (a per-lane pointer keeps it out of
    // the scalar registers, which the wide instances have none to spare of)
    const bool has_memo = f.memo != nullptr && q1 > q0;   // an empty chunk holds no piece
    AT* mlane = has_memo ? (AT*)f.memo + (int64_t)f.pid_base[ch] * f.Ks + lane : nullptr;
    auto fold = [&]() __attribute__((always_inline)) {
        if (has_memo) {   // wave-uniform
#pragma unroll
            for (int j = 0; j < KSL; ++j)
                if (lane + 64 * j < f.Ks) mlane[64 * j] = sacc[j];
            mlane += f.Ks;
        }
#pragma unroll
        for (int j = 0; j < KSL; ++j) {
#pragma unroll
            for (int r = 0; r < RF; ++r) yacc[j][r] += sacc[j] * u[r];
            sacc[j] = AT(0);
        }
    };
    auto flush_row = [&]() __attribute__((always_inline)) {
        const bool owner = (srow != s0) || (slot < 0);
        // select the base as an integer (a pointer select here was lowered through scratch)
        const uint64_t base = owner ? (uint64_t)(uintptr_t)a.Y : (uint64_t)(uintptr_t)a.carry;
        const int64_t row0 = owner ? (int64_t)ld_const(a.rows, srow) * K : (int64_t)slot * K;
        AT* dst = (AT*)(uintptr_t)base + row0;
#pragma unroll
        for (int j = 0; j < KSL; ++j) {
            const int cs = lane + 64 * j;
            if (cs < f.Ks) {
#pragma unroll
                for (int r = 0; r < RF; ++r)
                    if (r < Rf) dst[(int64_t)cs * Rf + r] = yacc[j][r];
            }
#pragma unroll
            for (int r = 0; r < RF; ++r) yacc[j][r] = AT(0);
        }
        if (owner) zero_gaps<AT>(a, srow, lane);
    };

    load_idx(q0, i1, x1);
    if (q0 + 64 < q1) load_idx(q0 + 64, i2, x2);
    load_rows(i1);
    for (int p = q0; p < q1; p += 64) {
        const int n = min(64, q1 - p);
        const bool valid = lane < n;
        // stage this batch: its rows (loaded one batch ago) into the LDS slot
        const int iflag = (valid && i1[0] < 0) ? 1 : 0;
        const int ifib = i1[NM1 - 1];
        Tx[lane] = valid ? x1 : AT(0);
        {
            int kin = 0;
#pragma unroll
            for (int t = 0; t < NM1; ++t) {
                const ST* vals = (const ST*)raw[t];
                if (t == NM1 - 1) {
#pragma unroll
                    for (int r = 0; r < RF; ++r)
                        Tuf[lane * RF + r] = (r < Rf && r < LDC) ? load_as<AT, ST>(vals, (int64_t)(r < LDC ? r : 0)) : AT(0);
                } else {
                    const int R = f.Rin[kin], o = f.off[kin];
#pragma unroll
                    for (int r = 0; r < LDC; ++r)
                        if (r < R) Tin[(o + r) * kFiberStride + lane] = load_as<AT, ST>(vals, (int64_t)r);
                    ++kin;
                }
            }
        }
        // fiber and row starts of this batch
        int prev = __shfl_up(ifib, 1);
        if (lane == 0) prev = prev_if;
        const uint64_t rstart = __ballot(iflag);
        const uint64_t fstart = __ballot(valid && (iflag || ifib != prev));
        prev_if = __shfl(ifib, n - 1);
        // prefetch: rows of the next batch, indices of the one after
        if (p + 64 < q1) {
            i1 = i2;
            x1 = x2;
            load_rows(i1);
            if (p + 128 < q1) load_idx(p + 128, i2, x2);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // walk the batch, four nonzeros at a time (n is a multiple of 4)
        for (int t0 = 0; t0 < n; t0 += 4) {
            const at4 xv = *(const at4*)&Tx[t0];
            at4 pr[KSL];
#pragma unroll
            for (int j = 0; j < KSL; ++j) {
                at4 v = xv;
#pragma unroll
                for (int k = 0; k < NM1 - 1; ++k) v *= *(const at4*)&Tin[toff[j][k] * kFiberStride + t0];
                pr[j] = v;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int t = t0 + e;
                const bool first = (p + t == q0);
                if (((fstart >> t) & 1ull) || first) {
                    if (!first) fold();
                    if (((rstart >> t) & 1ull) && !first) {
                        flush_row();
                        ++srow;
                    }
#pragma unroll
                    for (int r = 0; r < RF; r += 4) {
                        const at4 uv = *(const at4*)&Tuf[t * RF + r];
                        u[r] = uv.x; u[r + 1] = uv.y; u[r + 2] = uv.z; u[r + 3] = uv.w;
                    }
                }
#pragma unroll
                for (int j = 0; j < KSL; ++j) sacc[j] += pr[j][e];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    fold();
    flush_row();
}

// Adds the carry slots of each split row, in slot order, to the row written by its owner.  The
// loads are issued eight slots at a time (a hot row can span hundreds of pieces); the additions
// keep slot order.
template <typename AT>
__global__ __launch_bounds__(256) void k_ttmc_fixup(const int32_t* __restrict__ split,
                                                    const int32_t* __restrict__ rows, int K,
                                                    const AT* __restrict__ carry, AT* __restrict__ Y) {
    const int sp = blockIdx.x;
    const int s = split[3 * sp], f = split[3 * sp + 1], l = split[3 * sp + 2];
    AT* y = Y + (int64_t)rows[s] * K;
    for (int c = threadIdx.x; c < K; c += blockDim.x) {
        AT acc = AT(0);
        int k = f;
        for (; k + 8 <= l + 1; k += 8) {
            AT v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = carry[(int64_t)(k + u) * K + c];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u];
        }
        for (; k <= l; ++k) acc += carry[(int64_t)k * K + c];
        y[c] += acc;
    }
}

template <typename AT, typename ST>
int launch_generic(const TtmcArgs& a, hipStream_t s) {
    unsigned grid = (unsigned)((a.nchunks + 3) / 4);
    size_t lds = (size_t)a.K * a.nm1 * sizeof(uint16_t);
    int kpl = (a.K + 63) / 64;
#define TK_GEN(KP)                                                                      \
    k_ttmc_generic<AT, ST, KP><<<grid, 256, lds, s>>>(a);                               \
    TK_LAUNCH_CHECK("k_ttmc_generic");                                                  \
    return TK_OK;
    if (kpl <= 1) { TK_GEN(1) }
    if (kpl <= 2) { TK_GEN(2) }
    if (kpl <= 4) { TK_GEN(4) }
    if (kpl <= 8) { TK_GEN(8) }
    if (kpl <= 16) { TK_GEN(16) }
    if (kpl <= 32) { TK_GEN(32) }
    TK_GEN(64)
#undef TK_GEN
}

template <typename AT, typename ST, int NM1>
int launch_fiber_typed(const TtmcArgs& a, const FiberArgs& f, int ldc, hipStream_t s) {
    const unsigned grid = (unsigned)((a.nchunks + 3) / 4);
    const int ksl = (f.Ks + 63) / 64;
#define TK_FIB(KSL, RF, LDC)                                                                   \
    {                                                                                          \
        const size_t lds = (size_t)4 * fiber_slot_words<AT, RF>(f.tw) * sizeof(AT);            \
        k_ttmc_fiber<AT, ST, NM1, KSL, RF, LDC><<<grid, 256, lds, s>>>(a, f);                  \
        TK_LAUNCH_CHECK("k_ttmc_fiber");                                                       \
        return TK_OK;                                                                          \
    }
    if (ldc == 8) {   // every rank <= 8: 8-column factor copies
        if (ksl <= 1) TK_FIB(1, 8, 8)
        if (ksl <= 2) TK_FIB(2, 8, 8)
        if (ksl <= 4) TK_FIB(4, 8, 8)
        TK_FIB(8, 8, 8)
    }
    if (f.Rf <= 8) {
        if (ksl <= 1) TK_FIB(1, 8, 16)
        if (ksl <= 2) TK_FIB(2, 8, 16)
        if (ksl <= 4) TK_FIB(4, 8, 16)
        TK_FIB(8, 8, 16)
    }
    if (ksl <= 1) TK_FIB(1, 16, 16)
    if (ksl <= 2) TK_FIB(2, 16, 16)
    TK_FIB(4, 16, 16)
#undef TK_FIB
}

template <int NM1>
int launch_fiber_n(int dtype, const TtmcArgs& a, const FiberArgs& f, int ldc, hipStream_t s) {
    if (dtype == TK_F64) return launch_fiber_typed<double, double, NM1>(a, f, ldc, s);
    if (dtype == TK_F32) return launch_fiber_typed<float, float, NM1>(a, f, ldc, s);
    return launch_fiber_typed<float, bf16_t, NM1>(a, f, ldc, s);
}

int launch_fiber(int dtype, const TtmcArgs& a, const FiberArgs& f, int ldc, hipStream_t s) {
    if (a.nm1 == 3) return launch_fiber_n<3>(dtype, a, f, ldc, s);
    return launch_fiber_n<4>(dtype, a, f, ldc, s);
}

}  // namespace

int factor_ld(int N, const int32_t* ranks, int t) {
    bool narrow = N >= 4;
    for (int k = 0; k < N; ++k) narrow = narrow && ranks[k] <= 8;
    return narrow ? 8 : pad_rank(ranks[t]);
}

int ttmc_kernel_for(int N, const int64_t* dims, const int32_t* ranks, int dtype, int mode) {
    int others[kMaxOrder - 1], no = 0;
    for (int t = 0; t < N; ++t)
        if (t != mode) others[no++] = t;
    if (N == 3) {
        bool ok = true;
        for (int j = 0; j < 2; ++j) {
            const int t = others[j];
            const int ld = factor_ld(N, ranks, t);
            // the order-3 kernels form gather offsets in 32 bits (byte offsets in k_ttmc3_lds,
            // element offsets in int in k_ttmc3_mfma): only factors below 2^31 bytes take them
            const bool off32 = (uint64_t)dims[t] * (uint64_t)ld * dtype_size(dtype) < (1ull << 31);
            ok = ok && ranks[t] <= 16 && ld == 16 && off32;
        }
        return ok ? TK_TTMC_ORDER3 : TK_TTMC_GENERIC;
    }
    if (N == 4 || N == 5) {
        // fiber mode = the last other mode; inner modes the others
        int off = 0, Ks = 1;
        bool ok = true;
        for (int k = 0; k < N - 2; ++k) {
            ok = ok && ranks[others[k]] <= 16;
            off += ranks[others[k]];
            Ks *= ranks[others[k]];
        }
        for (int j = 0; j < N - 1; ++j) {
            const int ld = factor_ld(N, ranks, others[j]);
            ok = ok && (ld == 8 || ld == 16);
        }
        const int Rf = ranks[others[N - 2]];
        ok = ok && off <= kFiberTile && ((Rf <= 8 && Ks <= 64 * 8) || (Rf <= 16 && Ks <= 64 * 4));
        return ok ? TK_TTMC_FIBER : TK_TTMC_GENERIC;
    }
    return TK_TTMC_GENERIC;
}

namespace {

TtmcArgs mode_args(tk_ctx* ctx, int mode, void* Y, const void* val) {
    const ModeLayout& ml = ctx->mode[mode];
    const int N = ctx->N;
    TtmcArgs a{};
    a.chunk_ptr = ml.chunk_ptr;
    a.chunk_row = ml.chunk_row;
    a.chunk_slot = ml.chunk_slot;
    a.nchunks = (int32_t)ml.nchunks;
    a.ptr = ml.pptr;
    a.rows = ml.rows;
    a.S = (int32_t)ml.S;
    a.In = (int32_t)ctx->dims[mode];
    a.idx = ml.idx;
    a.nnz = ml.P;
    a.val = val ? val : ml.val;
    a.nm1 = N - 1;
    a.K = (int32_t)ml.K;
    a.Y = Y;
    a.carry = ctx->ws.carry;
    for (int j = 0; j < N - 1; ++j) {
        int t = ml.others[j];
        a.F[j] = ctx->Ulp[t];
        a.ld[j] = ctx->ldU[t];
        a.R[j] = ctx->ranks[t];
    }
    return a;
}

int run_fixup(tk_ctx* ctx, const ModeLayout& ml, void* Y, hipStream_t s) {
    if (ml.nsplit > 0) {
        if (ctx->dtype == TK_F64)
            k_ttmc_fixup<double><<<(unsigned)ml.nsplit, 256, 0, s>>>(ml.split, ml.rows, (int)ml.K,
                                                                     (const double*)ctx->ws.carry, (double*)Y);
        else
            k_ttmc_fixup<float><<<(unsigned)ml.nsplit, 256, 0, s>>>(ml.split, ml.rows, (int)ml.K,
                                                                    (const float*)ctx->ws.carry, (float*)Y);
        TK_LAUNCH_CHECK("k_ttmc_fixup");
    }
    return TK_OK;
}

}  // namespace

bool ttmc_residual_form(const tk_ctx* ctx, int mode) {
    return ctx->N == 3 && ctx->dtype == TK_F32 &&
           ttmc_kernel_for(ctx->N, ctx->dims, ctx->ranks, ctx->dtype, mode) == TK_TTMC_ORDER3;
}

int ttmc_residual_run(tk_ctx* ctx, int mode, void* Y, const float* W, double* part, hipStream_t s) {
    const ModeLayout& ml = ctx->mode[mode];
    if (!ttmc_residual_form(ctx, mode))
        return set_error(TK_ERR_ARG, "residual TTMc: mode %d does not take the order-3 FP32 kernel", mode);
    if (ml.nchunks == 0) return fill_zero(Y, (size_t)ctx->dims[mode] * ml.K * sizeof(float), s);
    const TtmcArgs a = mode_args(ctx, mode, Y, nullptr);
    ResArgs r{W, part};
    k_ttmc3_lds<float, true><<<(unsigned)((ml.nchunks + 3) / 4), 256, 0, s>>>(a, r);
    TK_LAUNCH_CHECK("k_ttmc3_lds");
    return run_fixup(ctx, ml, Y, s);
}

int ttmc_run(tk_ctx* ctx, int mode, void* Y, hipStream_t s, hipEvent_t* ev_main, const void* val, void* memo,
             const int32_t* pid_base) {
    const ModeLayout& ml = ctx->mode[mode];
    const int N = ctx->N;
    const int64_t In = ctx->dims[mode];
    const size_t ysz = ytype_size(ctx->dtype);
    if (ml.nchunks == 0) {
        if (ev_main) TK_HIP(hipEventRecord(ev_main[0], s));
        const int st0 = fill_zero(Y, (size_t)In * ml.K * ysz, s);
        if (ev_main) TK_HIP(hipEventRecord(ev_main[1], s));
        return st0;
    }
    TtmcArgs a = mode_args(ctx, mode, Y, val);
    const int kernel = ttmc_kernel_for(N, ctx->dims, ctx->ranks, ctx->dtype, mode);
    const bool mfma_ok = kernel == TK_TTMC_ORDER3;
    const unsigned grid = (unsigned)((ml.nchunks + 3) / 4);
    int st = TK_OK;
    // fiber-factored kernel for order >= 4 (fiber mode = last other mode)
    FiberArgs fa{};
    bool fiber_ok = kernel == TK_TTMC_FIBER && ml.fiber_slot == N - 2;
    if (fiber_ok) {
        fa.nin = N - 2;
        int off = 0;
        fa.Ks = 1;
        bool small = true;   // every staged row fits the 16 loaded columns
        for (int k = 0; k < N - 2; ++k) {
            small = small && a.R[k] <= 16;
            fa.off[k] = off;
            fa.Rin[k] = a.R[k];
            off += a.R[k];
            fa.Ks *= a.R[k];
        }
        fa.Rf = a.R[N - 2];
        fa.tw = off;
        fa.memo = memo;
        fa.pid_base = pid_base;
        fiber_ok = small;   // always true when ttmc_kernel_for chose this kernel
    }
    if (memo && !fiber_ok) return set_error(TK_ERR_ARG, "fiber sums requested from a mode without the fiber kernel");
    if (ev_main) TK_HIP(hipEventRecord(ev_main[0], s));
    if (mfma_ok) {
        if (ctx->dtype == TK_F64) {
            k_ttmc3_mfma<double, double><<<grid, 256, 0, s>>>(a);
            TK_LAUNCH_CHECK("k_ttmc3_mfma");
        } else if (ctx->dtype == TK_F32) {
            k_ttmc3_lds<float, false><<<grid, 256, 0, s>>>(a, ResArgs{});
            TK_LAUNCH_CHECK("k_ttmc3_lds");
        } else {
            k_ttmc3_bf<<<grid, 256, 0, s>>>(a);
            TK_LAUNCH_CHECK("k_ttmc3_bf");
        }
    } else if (fiber_ok) {
        // factor copies of 8 columns (every rank <= 8) or 16
        int ldc = 8;
        for (int j = 0; j < N - 1; ++j) ldc = (a.ld[j] == 8) ? ldc : 16;
        st = launch_fiber(ctx->dtype, a, fa, ldc, s);
        if (st) return st;
    } else {
        if (ctx->dtype == TK_F64) st = launch_generic<double, double>(a, s);
        else if (ctx->dtype == TK_F32) st = launch_generic<float, float>(a, s);
        else st = launch_generic<float, bf16_t>(a, s);
        if (st) return st;
    }
    if (ev_main) TK_HIP(hipEventRecord(ev_main[1], s));
    return run_fixup(ctx, ml, Y, s);
}

}  // namespace tk
