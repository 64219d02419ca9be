// march_rows.h -- the radiance-interval march + merge kernel (Osborne &
// Sannikov, arXiv:2408.14425, Secs. 2.2-2.3 and 3.2), templated on how a ray
// step obtains its opacity and source function (Op) and on what happens with
// the merged radiance (Epi).
//
// A wavefront holds 4 rays x 16 wavelengths: each 16-lane row is one ray of
// one 16-wavelength batch (or of two batches, Op::kW = 2, each lane holding
// wavelength l of both). The cell walk is cooperative per row: lane j
// computes the one or two segments of the j-th grid column the ray crosses
// along its major axis (plane crossings in FP64, so cell boundaries are
// exact), the row compacts them into LDS, and all 16 wavelength lanes then
// step through the list with the FP32 radiative update
//   I += T S (1 - 2^{-y}),  T *= 2^{-y},  y = optical depth in log2 units,
// front to back, which equals the back-to-front piecewise-constant solution
// of Sec. 3.2. The merge with the cascade above (Sec. 2.3.1) follows:
//   Itilde = I + T * sum_taps w_x w_z (1/4) sum_j Itilde_up(tap, 4k + j).
// In k_march_shared the 4 rows are 4 probes of one direction and one walk
// of 64 columns serves all four (walk_ray_shared), with the same segments.
#pragma once

#include "rcx_internal.h"

namespace rcx {
namespace march {

constexpr int kBlock = 256;                       // 4 wavefronts
constexpr int kRaysPerBlock = (kBlock / 64) * 4;  // 4 rows of 16 lanes per wavefront
constexpr int kLB = 16;                           // wavelengths per batch = lanes per row
constexpr unsigned kXcds = 8;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// Workgroups are dispatched round-robin over the 8 XCDs. XCD x takes
// chunks of `chunk` consecutive logical blocks, chunk i on XCD i mod 8:
// all XCDs advance through the ray order together (they share the field data
// in the Infinity Cache) while each works on compact groups of rays (shared
// in its own L2). The tail that does not fill 8 whole chunks keeps the
// identity order. The chunk is a launch parameter (LevelDesc::xcd_chunk,
// chosen by the autotuner; 128 by default).
constexpr unsigned kXcdChunk = 128;
__device__ __forceinline__ unsigned xcd_block_chunked(unsigned b, unsigned nb, unsigned chunk = kXcdChunk)
{
    const unsigned full = nb / (kXcds * chunk) * (kXcds * chunk);
    if (b >= full) return b;
    const unsigned x = b % kXcds, slot = b / kXcds;
    return (slot / chunk) * (kXcds * chunk) + x * chunk + slot % chunk;
}
// The same with the chunk a launch constant of the cascade (its divisions
// precomputed in LevelDesc::dec).
__device__ __forceinline__ unsigned xcd_block_chunked(unsigned b, unsigned nb, const LevelDesc::Decode& D)
{
    const unsigned c8 = D.chunk8.d, full = D.chunk8.div(nb) * c8;
    if (b >= full) return b;
    const unsigned x = b % kXcds, slot = b / kXcds;
    const unsigned q = D.chunk.div(slot);
    return q * c8 + x * D.chunk.d + (slot - q * D.chunk.d);
}

// 1 - 2^{-y} (e = 2^{-y}) as the smaller of the three-term series (an upper
// bound of it for every y >= 0: the remainder's derivative is non-negative)
// and (1 + 2^-22) - 2^{-y} (the offset keeps the cancelling form above the
// series where the series is the better one), with no compare and select:
// at most 6e-6 relative, 0 at y = 0.
__device__ __forceinline__ float one_minus_exp2_neg_min(float y, float e)
{
    constexpr float c1 = 0.6931471805599453f;  // ln 2
    constexpr float c2 = 0.2402265069591007f;  // (ln 2)^2 / 2
    constexpr float c3 = 0.0555041086648216f;  // (ln 2)^3 / 6
    const float ser = y * (c1 - y * (c2 - y * c3));
    return fminf(ser, (1.0f + 0x1p-22f) - e);
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Geometry of the ray a row marches.
struct RayInfo {
    int32_t k, u, v;  // direction, probe coordinates
    int64_t ray;      // ray index within the cascade
    double wx, wz;    // direction
    bool active;
};

// 16-bit cascade storage (RCX_STORE_F16_SCALED) of a non-negative
// radiance: FP32 rounded to FP16's 10-bit significand (to nearest, ties to
// even), its 8-bit exponent E rebased by the wavelength's bias eb into 6
// bits, code = (E - eb) 2^10 + significand. FP16's sign bit is spent on
// range (radiances are never negative): with eb = E(max S) - 62 the codes
// cover the 63 binades below 2^(E(max S) + 2 - 127) > 2 max S, every value
// there with FP16's relative rounding 2^-11; code 0 is 0, and values more
// than ~2^62 below max S flush to it. eb1024 = eb * 2^10.
__device__ __forceinline__ uint16_t enc_h16(float x, int32_t eb1024)
{
    const uint32_t u = __float_as_uint(x) & 0x7FFFFFFFu;
    const int32_t r = (int32_t)((u + 0x0FFFu + ((u >> 13) & 1u)) >> 13) - eb1024;
    return (uint16_t)min(max(r, 0), 0xFFFF);
}
__device__ __forceinline__ float dec_h16(uint32_t c, int32_t eb1024)
{
    const float v = __uint_as_float((uint32_t)((int32_t)c + eb1024) << 13);
    return c != 0u ? v : 0.0f;
}

// Readers of the merged cascade above: FP32, or the 16-bit codes with a
// per-wavelength exponent bias. Slot w = 1 (a second wavelength batch
// marched by the same lanes) lies `stride` elements after slot 0, with the
// next batch's biases.
struct UpF32 {
    const float* p;
    int64_t stride = 0;
    __device__ __forceinline__ void init(int) {}
    __device__ __forceinline__ float get(int64_t i, int w) const { return p[i + w * stride]; }
};
struct UpF16 {
    const uint16_t* p;
    const int32_t* ebias_b;  // [16] of this batch (then [16] of the next when stride != 0)
    int64_t stride = 0;
    int32_t B = 0, B2 = 0;   // the lane's biases * 2^10
    __device__ __forceinline__ void init(int l)
    {
        B = ebias_b[l] * 1024;
        if (stride != 0) B2 = ebias_b[l + kLB] * 1024;
    }
    __device__ __forceinline__ float get(int64_t i, int w) const { return dec_h16(p[i + w * stride], w ? B2 : B); }
};

// W slots `stride` elements apart, slot w with the biases of batch b + w
// (ebias_b[w * 16 + l]): the cascades of W batches of one line marched
// together.
// The biases are read where a merge needs them (entry i belongs to lane
// i mod 16), so no register holds them during the march.
template <int W>
struct UpF16Slots {
    const uint16_t* p;
    const int32_t* ebias_b;  // [W][16]
    int64_t stride = 0;
    __device__ __forceinline__ void init(int) {}
    __device__ __forceinline__ float get(int64_t i, int w) const
    {
        return dec_h16(p[i + w * stride], ebias_b[(int)(i & (kLB - 1)) + w * kLB] * 1024);
    }
};

// Lane state shared by the kernels that march rows of rays.
struct RowCtx {
    int lane, w, row, l;
    uint64_t row_bits, lt_bits;
};

__device__ __forceinline__ RowCtx row_ctx()
{
    RowCtx c;
    c.lane = threadIdx.x & 63;
    c.w = threadIdx.x >> 6;
    c.row = c.lane >> 4;
    c.l = c.lane & 15;
    c.row_bits = 0xFFFFull << (16 * c.row);
    c.lt_bits = (c.lane == 0) ? 0ull : (~0ull >> (64 - c.lane));
    return c;
}

// Segments per row and chunk: 16 columns, at most two segments each.
constexpr int kSegs = 32;
// LDS rows of the segment lists (16 uint4 = 32 entries) and of the staged
// data, each padded by one element: the 4 rows of a wavefront read 4
// different addresses in the same instruction, and unpadded (256 or 1024
// bytes apart) they would fall in the same banks.
constexpr int kSegRow = 17;
constexpr int kStgRow = kSegs + 1;

// One front-to-back step: f = {optical depth per cell in log2 units, S},
// ds the segment length in cells.
__device__ __forceinline__ void step(float2 f, float ds, float& I, float& T)
{
    const float y = f.x * ds;
    const float e = __builtin_amdgcn_exp2f(-y);
    I = fmaf(T * f.y, one_minus_exp2_neg_min(y, e), I);
    T *= e;
}

// Plane crossings. A ray line from c = k + f per axis (k = floor(c), f =
// c - k, both exact) meets plane X at t = ((X - k) - f) / w: X - k is an
// exact integer and, for probe centres (f = 0 or 1/2), so is its difference
// with f, so t takes one rounding and is the same for every start point
// moved by whole cells. Walks from probes whole cells apart therefore find
// bitwise the same segments (walk_ray_shared relies on it), and the
// crossing of the domain's exit plane equals the clip bound exactly.
__device__ __forceinline__ double plane_t(double X, double k, double f, double inv_w)
{
    return ((X - k) - f) * inv_w;
}

// A step of known optical depth y = f.x (log2 units), for the staged
// marches (the segment length is folded into their records).
__device__ __forceinline__ void step_unit(float2 f, float& I, float& T)
{
    const float y = f.x;
    const float e = __builtin_amdgcn_exp2f(-y);
    I = fmaf(T * f.y, one_minus_exp2_neg_min(y, e), I);
    T *= e;
}

// Walk one ray per row: the segments of the line (cx, cz) + t (wx, wz),
// t in [t_lo, t_hi), that lie in the domain (d = {wx, wz, 1/wx, 1/wz}),
// stepped front to back into I and T (Op::kW slots per lane). Rows with walk
// false step through nothing but still take part in the wavefront-wide
// ballots.
// An Op whose step data depends on the cell only (the same for all 16
// wavelength lanes of a row) sets kStaged: the lane that finds a segment
// loads that data once (Op::stage_load, then Op::stage_make forms the
// entry with the segment's length folded in) in place of a segment-list
// entry, and the step loop reads it back from LDS (stg, this wavefront's
// [4 rows][kSegs] entries) instead of issuing a dependent global load per
// step; Op::resolve4 turns a group of 4 staged steps into {optical depth
// of the step, S}.
template <class Op>
__device__ __forceinline__ void walk_ray(const LevelDesc& L, int32_t nx, int32_t nz, Op& op, double cx, double cz,
                                         const double4 d, double t_lo, double t_hi, bool walk,
                                         uint4 (*seg)[kSegRow], typename Op::Stage (*stg)[kStgRow],
                                         const RowCtx& cx_, float (&I)[Op::kW], float (&T)[Op::kW])
{
    const int row = cx_.row, l = cx_.l;
    const uint64_t row_bits = cx_.row_bits, lt_bits = cx_.lt_bits;
    const double kx = floor(cx), kz = floor(cz), fx = cx - kx, fz = cz - kz;
    const double ax = plane_t(0.0, kx, fx, d.z), bx = plane_t((double)nx, kx, fx, d.z);
    const double az = plane_t(0.0, kz, fz, d.w), bz = plane_t((double)nz, kz, fz, d.w);
    double lo = fmax(t_lo, fmax(fmin(ax, bx), fmin(az, bz)));
    double hi = fmin(t_hi, fmin(fmax(ax, bx), fmax(az, bz)));
    if (!walk) {
        lo = 1.0;
        hi = 0.0;
    }

    // Major axis m (the one crossed at least as often), minor axis n.
    const bool xmaj = fabs(d.x) >= fabs(d.y);
    const double wm = xmaj ? d.x : d.y, wn = xmaj ? d.y : d.x;
    const double km = xmaj ? kx : kz, kn = xmaj ? kz : kx, fm = xmaj ? fx : fz, fn = xmaj ? fz : fx;
    const double im_ = xmaj ? d.z : d.w, in_ = xmaj ? d.w : d.z;
    const int nm = xmaj ? nx : nz, nn = xmaj ? nz : nx;
    const int strm = xmaj ? 1 : nx, strn = xmaj ? nx : 1;
    const int sm = wm > 0.0 ? 1 : -1, sn = wn > 0.0 ? 1 : -1;
    const int ikm = (int)km, ikn = (int)kn;

    // major-axis position at lo relative to km
    const double qm0 = fm + lo * wm;
    int im0 = ikm + (wm > 0.0 ? (int)floor(qm0) : (int)ceil(qm0) - 1);
    im0 = min(max(im0, 0), nm - 1);
    const int mfirst = wm > 0.0 ? im0 + 1 : im0;  // first m-plane crossed

    // kW wavelength batches per lane (slot w of lane l is wavelength l of
    // batch w): the walk and the segment list serve all of them
    constexpr int W = Op::kW;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        I[w] = 0.0f;
        T[w] = 1.0f;
    }
    const int max_chunks = (nm + 2 + 15) / 16 + 1;
    // Minor-axis cell of a crossing at kn + qn: kn + floor(qn) if sn > 0,
    // else kn + ceil(qn) - 1 = kn + ~floor(-qn); both as kn + (floor(sn * qn)
    // ^ nflip) (sn * qn is exact). The products below stay within 24 bits
    // (cell < 2^24).
    const double snd = (double)sn;
    const int nflip = sn > 0 ? 0 : -1, nadd = sn > 0 ? 1 : 0;
    for (int chunk = 0; chunk < max_chunks; ++chunk) {
        // ---- column j of this row's ray: one or two segments
        const int j = chunk * 16 + l;
        const int pj = mfirst + __mul24(j - 1, sm);  // m-plane entering column j
        const double ta = (j == 0) ? lo : plane_t((double)(pj - ikm), 0.0, fm, im_);
        const double tb_ = fmin(plane_t((double)(pj + sm - ikm), 0.0, fm, im_), hi);
        const bool valid = ta < hi;
        const int im = min(max(im0 + __mul24(j, sm), 0), nm - 1);
        const double qn = fn + ta * wn;
        int in0 = ikn + ((int)floor(snd * qn) ^ nflip);
        in0 = min(max(in0, 0), nn - 1);
        const int nnext = in0 + nadd;
        const double tn = plane_t((double)(nnext - ikn), 0.0, fn, in_);
        const bool two = valid && tn < tb_;
        const double tmid = fmax(tn, ta);
        const int in1 = min(max(in0 + sn, 0), nn - 1);
        const int cm_ = __mul24(im, strm);
        const uint32_t cell1 = (uint32_t)(cm_ + __mul24(in0, strn));
        const uint32_t cell2 = (uint32_t)(cm_ + __mul24(in1, strn));
        const float ds1 = (float)(fmax((two ? tmid : tb_) - ta, 0.0) * L.ds_scale);
        const float ds2 = (float)(fmax(tb_ - tmid, 0.0) * L.ds_scale);
        // staged data: loads issued here, used after the compaction below
        typename Op::StageIn st1{}, st2{};
        if constexpr (Op::kStaged) {
            if (valid) st1 = op.stage_load(cell1);
            if (two) st2 = op.stage_load(cell2);
        }

        const uint64_t b1 = __ballot(valid);
        if (b1 == 0) break;
        const uint64_t b2 = __ballot(two);
        const int pos = (int)__popcll(b1 & row_bits & lt_bits) + (int)__popcll(b2 & row_bits & lt_bits);
        // longest list of the 4 rows, from the wave-uniform ballots
        int n_max = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t rb = 0xFFFFull << (16 * q);
            n_max = max(n_max, (int)__popcll(b1 & rb) + (int)__popcll(b2 & rb));
        }
        n_max = __builtin_amdgcn_readfirstlane(n_max);
        // Null entries are written everywhere first and the row's segments
        // over them (the LDS executes one wavefront's writes in issue order),
        // so the step loop needs no bounds test.
        if constexpr (Op::kStaged) {
            // staged records with their segment length folded in
            // (Op::stage_make); a null record (zeros) is a step with no
            // opacity and no emission. No segment list is needed.
            stg[row][l] = typename Op::Stage{};
            stg[row][l + 16] = typename Op::Stage{};
            if (valid) stg[row][pos] = op.stage_make(st1, ds1);
            if (two) stg[row][pos + 1] = op.stage_make(st2, ds2);
        } else {
            // entries: the Op's key of the cell (a byte offset for per-lane
            // fields) and ds; a null entry has no data and ds = 0
            uint2* srow = reinterpret_cast<uint2*>(&seg[row][0]);
            srow[l] = make_uint2(Op::kNullKey, 0u);
            srow[l + 16] = make_uint2(Op::kNullKey, 0u);
            if (valid) srow[pos] = make_uint2(op.key(cell1), __float_as_uint(ds1));
            if (two) srow[pos + 1] = make_uint2(op.key(cell2), __float_as_uint(ds2));
        }
        wave_sync();

        // ---- step through the row's segments, 4 at a time. Positions past
        // the row's count are steps with no opacity and no emission.
        if constexpr (Op::kStaged) {
            // step data in LDS (no global loads to overlap), optical depths
            // per step already (f.x includes ds)
            for (int s = 0; s < n_max; s += 4) {
                typename Op::Raw raw[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) raw[q] = stg[row][s + q];
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    float2 f[4];
                    op.resolve4(raw, f, w);
#pragma unroll
                    for (int q = 0; q < 4; ++q) step_unit(f[q], I[w], T[w]);
                }
            }
        } else {
            // per-lane data: the 4 loads of a group are issued together (a
            // software pipeline across groups measured no faster); a list
            // ending 1 or 2 entries into a group ends with a group of 2
#pragma unroll
            for (int s = 0; s < kSegs; s += 4) {
                if (s >= n_max) break;
                if (n_max - s <= 2) {
                    const uint4 e01 = seg[row][s >> 1];
                    typename Op::Raw raw[2][W];
                    op.fetch_key(e01.x, raw[0]);
                    op.fetch_key(e01.z, raw[1]);
#pragma unroll
                    for (int w = 0; w < W; ++w) step(op.resolve(raw[0][w]), __uint_as_float(e01.y), I[w], T[w]);
#pragma unroll
                    for (int w = 0; w < W; ++w) step(op.resolve(raw[1][w]), __uint_as_float(e01.w), I[w], T[w]);
                    break;
                }
                const uint4 e01 = seg[row][s >> 1];
                const uint4 e23 = seg[row][(s >> 1) + 1];
                const uint32_t cells[4] = {e01.x, e01.z, e23.x, e23.z};
                const float dsv[4] = {__uint_as_float(e01.y), __uint_as_float(e01.w), __uint_as_float(e23.y),
                                      __uint_as_float(e23.w)};
                typename Op::Raw raw[4][W];
#pragma unroll
                for (int q = 0; q < 4; ++q) op.fetch_key(cells[q], raw[q]);
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int w = 0; w < W; ++w) step(op.resolve(raw[q][w]), dsv[q], I[w], T[w]);
            }
        }
        wave_sync();
    }
}

// Shared-direction walk (k_march_shared): the 4 rows of the
// wavefront march one direction from 4 probes whose centres lie whole cells
// apart (integral probe spacing). One cooperative walk, 64 columns per chunk
// in the frame of row 0's probe on an unbounded grid, serves all four: row
// r's cell of a segment is the reference cell moved by r's probe offset, a
// constant step of the cell key. The domain's planes are grid planes of that
// frame and plane_t gives their crossings bitwise as row r's own walk would,
// so each segment lies wholly inside or outside row r's clip range
// [lo_r, hi_r]; the inside ones are a contiguous run of the list, found per
// chunk from ballots, and the rest step with the null key (no opacity, no
// emission). Row r thus steps the segments walk_ray would give it, with the
// same lengths, in the same order (up to zero-length ones, which change
// nothing): the results are bitwise those of walk_ray. The walk covers the
// union of the four ranges; the per-row walk runs 4 walks of 16 columns in
// its place.
constexpr int kSegShared = 128;  // entries per wavefront and chunk: 64 columns, <= 2 each

__device__ __forceinline__ double uniform_d(double x)
{
    const uint64_t b = __double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <class Op>
__device__ __forceinline__ void walk_ray_shared(const LevelDesc& L, int32_t nx, int32_t nz, Op& op, int32_t u,
                                                int32_t v, const double4 d, bool walk, uint2* seg,
                                                const RowCtx& cx_, float (&I)[Op::kW], float (&T)[Op::kW])
{
    static_assert(!Op::kStaged, "the shared walk takes per-lane field ops");
    constexpr int W = Op::kW;
    const int lane = cx_.lane, row = cx_.row;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        I[w] = 0.0f;
        T[w] = 1.0f;
    }
    // this row's clip range, as in walk_ray; +inf/-inf when it walks nothing
    const double cx = (u + 0.5) * L.s, cz = (v + 0.5) * L.s;
    double lo, hi;
    {
        const double kx = floor(cx), kz = floor(cz), fx = cx - kx, fz = cz - kz;
        const double ax = plane_t(0.0, kx, fx, d.z), bx = plane_t((double)nx, kx, fx, d.z);
        const double az = plane_t(0.0, kz, fz, d.w), bz = plane_t((double)nz, kz, fz, d.w);
        lo = fmax(L.ta, fmax(fmin(ax, bx), fmin(az, bz)));
        hi = fmin(L.tb, fmin(fmax(ax, bx), fmax(az, bz)));
        if (!walk || !(lo < hi)) {
            lo = INFINITY;
            hi = -INFINITY;
        }
    }
    double lo_q[4], hi_q[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        lo_q[q] = uniform_d(__shfl(lo, 16 * q));
        hi_q[q] = uniform_d(__shfl(hi, 16 * q));
    }
    const double T0 = fmin(fmin(lo_q[0], lo_q[1]), fmin(lo_q[2], lo_q[3]));
    const double T1 = fmax(fmax(hi_q[0], hi_q[1]), fmax(hi_q[2], hi_q[3]));
    if (!(T0 < T1)) return;  // no row walks anything

    // reference frame: row 0's probe; row offsets in whole cells
    const int32_t u0 = __builtin_amdgcn_readfirstlane(u), v0 = __builtin_amdgcn_readfirstlane(v);
    const int32_t is = (int32_t)L.s;
    const double c0x = (u0 + 0.5) * L.s, c0z = (v0 + 0.5) * L.s;
    // row r's cell key = reference key + dkey (mod 2^32; exact for cells in the domain)
    const uint32_t dkey =
        ((uint32_t)((v - v0) * is) * (uint32_t)nx + (uint32_t)((u - u0) * is)) * (uint32_t)(kLB * 8);

    const double k0x = floor(c0x), k0z = floor(c0z), fx = c0x - k0x, fz = c0z - k0z;
    const bool xmaj = fabs(d.x) >= fabs(d.y);
    const double wm = xmaj ? d.x : d.y, wn = xmaj ? d.y : d.x;
    const double fm = xmaj ? fx : fz, fn = xmaj ? fz : fx;
    const int ikm = (int)(xmaj ? k0x : k0z), ikn = (int)(xmaj ? k0z : k0x);
    const double im_ = xmaj ? d.z : d.w, in_ = xmaj ? d.w : d.z;
    const uint32_t kstrm = xmaj ? (uint32_t)(kLB * 8) : (uint32_t)nx * (kLB * 8);
    const uint32_t kstrn = xmaj ? (uint32_t)nx * (kLB * 8) : (uint32_t)(kLB * 8);
    const int sm = wm > 0.0 ? 1 : -1, sn = wn > 0.0 ? 1 : -1;
    // the same arithmetic as walk_ray, unclamped (cells outside the domain
    // belong to no row's range)
    const double qm0 = fm + T0 * wm;
    const int im0 = ikm + (wm > 0.0 ? (int)floor(qm0) : (int)ceil(qm0) - 1);
    const int mfirst = wm > 0.0 ? im0 + 1 : im0;
    const double snd = (double)sn;
    const int nflip = sn > 0 ? 0 : -1, nadd = sn > 0 ? 1 : 0;
    // columns crossed: at most (T1 - T0) |wm| + 2
    const int max_chunks = (int)((T1 - T0) * fabs(wm) * (1.0 / 64.0)) + 2;

    for (int chunk = 0; chunk < max_chunks; ++chunk) {
        const int j = chunk * 64 + lane;
        const int pj = mfirst + (j - 1) * sm;
        const double ta = (j == 0) ? T0 : plane_t((double)(pj - ikm), 0.0, fm, im_);
        const double tb_ = fmin(plane_t((double)(pj + sm - ikm), 0.0, fm, im_), T1);
        const bool valid = ta < T1;
        const int im = im0 + j * sm;
        const double qn = fn + ta * wn;
        const int in0 = ikn + ((int)floor(snd * qn) ^ nflip);
        const double tn = plane_t((double)(in0 + nadd - ikn), 0.0, fn, in_);
        const bool two = valid && tn < tb_;
        const double tmid = fmax(tn, ta);
        const double tend1 = two ? tmid : tb_;
        const uint32_t key1 = (uint32_t)im * kstrm + (uint32_t)in0 * kstrn;
        const uint32_t key2 = key1 + (sn > 0 ? kstrn : 0u - kstrn);
        const float ds1 = (float)(fmax(tend1 - ta, 0.0) * L.ds_scale);
        const float ds2 = (float)(fmax(tb_ - tmid, 0.0) * L.ds_scale);

        const uint64_t b1 = __ballot(valid);
        if (b1 == 0) break;
        const uint64_t b2 = __ballot(two);
        const int pos = (int)__popcll(b1 & cx_.lt_bits) + (int)__popcll(b2 & cx_.lt_bits);
        const int n = (int)__builtin_amdgcn_readfirstlane((int)__popcll(b1) + (int)__popcll(b2));
        // each row's run [a_q, e_q) of the list: a_q entries start before
        // lo_q, e_q end at or before hi_q (row q's clip bounds are crossings
        // of this walk, bitwise, so no segment straddles them)
        int a_q[4], e_q[4];
        bool full = true;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a_q[q] = (int)__popcll(__ballot(valid && ta < lo_q[q])) + (int)__popcll(__ballot(two && tmid < lo_q[q]));
            e_q[q] = (int)__popcll(__ballot(valid && tend1 <= hi_q[q])) + (int)__popcll(__ballot(two && tb_ <= hi_q[q]));
            full = full && a_q[q] == 0 && e_q[q] == n;
        }
        const int a = row == 0 ? a_q[0] : row == 1 ? a_q[1] : row == 2 ? a_q[2] : a_q[3];
        const int e = row == 0 ? e_q[0] : row == 1 ? e_q[1] : row == 2 ? e_q[2] : e_q[3];
        const uint32_t len = (uint32_t)max(e - a, 0);
        // null entries first, then the list (one wavefront's LDS writes
        // execute in issue order)
        seg[lane] = make_uint2(Op::kNullKey, 0u);
        seg[lane + 64] = make_uint2(Op::kNullKey, 0u);
        if (valid) seg[pos] = make_uint2(key1, __float_as_uint(ds1));
        if (two) seg[pos + 1] = make_uint2(key2, __float_as_uint(ds2));
        wave_sync();

        const uint4* seg4 = reinterpret_cast<const uint4*>(seg);
        for (int s = 0; s < n; s += 4) {
            const uint4 e01 = seg4[s >> 1];
            const uint4 e23 = seg4[(s >> 1) + 1];
            const uint32_t keys[4] = {e01.x, e01.z, e23.x, e23.z};
            const float dsv[4] = {__uint_as_float(e01.y), __uint_as_float(e01.w), __uint_as_float(e23.y),
                                  __uint_as_float(e23.w)};
            typename Op::Raw raw[4][W];
            if (full && s + 4 <= n) {
#pragma unroll
                for (int q = 0; q < 4; ++q) op.fetch_key(keys[q] + dkey, raw[q]);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    op.fetch_key((uint32_t)(s + q - a) < len ? keys[q] + dkey : Op::kNullKey, raw[q]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int w = 0; w < W; ++w) step(op.resolve(raw[q][w]), dsv[q], I[w], T[w]);
        }
        wave_sync();
    }
}

// Merge the marched (I, T) of one row's ray with the cascade above and
// hand it to the epilogue.
template <class Op, class Epi, class Up>
__device__ __forceinline__ void merge_finish(const LevelDesc& L, Op& op, Epi& epi, const Up& up, const RayInfo& ri,
                                             int l, int lane, float (&I)[Op::kW], const float (&T)[Op::kW])
{
    constexpr int W = Op::kW;
    if (ri.active && L.has_up) {
        // Bilinear taps on the cascade above: q = (u + 1/2)/2 - 1/2, so
        // even u -> taps (u/2 - 1, u/2) with weights (1/4, 3/4), odd u ->
        // taps ((u-1)/2, (u+1)/2) with weights (3/4, 1/4); clamped.
        const int bx0 = (ri.u - 1) >> 1, bz0 = (ri.v - 1) >> 1;
        const float fx = (ri.u & 1) ? 0.25f : 0.75f;
        const float fz = (ri.v & 1) ? 0.25f : 0.75f;
        const int txs[2] = {min(max(bx0, 0), L.qx - 1), min(max(bx0 + 1, 0), L.qx - 1)};
        const int tzs[2] = {min(max(bz0, 0), L.qz - 1), min(max(bz0 + 1, 0), L.qz - 1)};
        const float wxs[2] = {1.0f - fx, fx};
        const float wzs[2] = {1.0f - fz, fz};
        float far[W];
#pragma unroll
        for (int w = 0; w < W; ++w) far[w] = 0.0f;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) {
                const int64_t bi = (((int64_t)tzs[a] * L.qx + txs[bb]) * L.nd_up + 4 * (int64_t)ri.k) * kLB + l;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const float c4 =
                        up.get(bi, w) + up.get(bi + kLB, w) + up.get(bi + 2 * kLB, w) + up.get(bi + 3 * kLB, w);
                    far[w] = fmaf(wzs[a] * wxs[bb], 0.25f * c4, far[w]);
                }
            }
#pragma unroll
        for (int w = 0; w < W; ++w) I[w] = fmaf(T[w], far[w], I[w]);
    }
    if constexpr (W == 1) {
        epi.finish(ri, l, lane, I[0], op);
    } else {
        epi.finish_slots(ri, l, lane, I, op);
    }
}

// March, merge and finish one ray per row. ray = output index of the ray
// in its cascade, (u, v, k) its probe and direction; active false for rows
// past the end (they still take part in the wavefront-wide ballots).
template <class Op, class Epi, class Up>
__device__ __forceinline__ void march_ray(const LevelDesc& L, int32_t nx, int32_t nz, Op& op, Epi& epi,
                                          const double4* __restrict__ dirs, const Up& up, uint4 (*seg)[kSegRow],
                                          typename Op::Stage (*stg)[kStgRow], const RowCtx& cx_, int64_t ray,
                                          int32_t u, int32_t v, int32_t k, bool active)
{
    const int lane = cx_.lane, l = cx_.l;
    RayInfo ri;
    ri.ray = ray;
    ri.active = active;
    ri.k = k;
    ri.u = u;
    ri.v = v;

    const double cx = (ri.u + 0.5) * L.s, cz = (ri.v + 0.5) * L.s;
    const double4 d = dirs[ri.k];  // {wx, wz, 1/wx, 1/wz}
    ri.wx = d.x;
    ri.wz = d.y;
    op.begin_ray(d.x, d.y);
    constexpr int W = Op::kW;
    float I[W], T[W];
    walk_ray(L, nx, nz, op, cx, cz, d, L.ta, L.tb, ri.active, seg, stg, cx_, I, T);

    if (ri.active && L.has_up) {
        // Bilinear taps on the cascade above: q = (u + 1/2)/2 - 1/2, so
        // even u -> taps (u/2 - 1, u/2) with weights (1/4, 3/4), odd u ->
        // taps ((u-1)/2, (u+1)/2) with weights (3/4, 1/4); clamped.
        const int bx0 = (ri.u - 1) >> 1, bz0 = (ri.v - 1) >> 1;
        const float fx = (ri.u & 1) ? 0.25f : 0.75f;
        const float fz = (ri.v & 1) ? 0.25f : 0.75f;
        const int txs[2] = {min(max(bx0, 0), L.qx - 1), min(max(bx0 + 1, 0), L.qx - 1)};
        const int tzs[2] = {min(max(bz0, 0), L.qz - 1), min(max(bz0 + 1, 0), L.qz - 1)};
        const float wxs[2] = {1.0f - fx, fx};
        const float wzs[2] = {1.0f - fz, fz};
        float far[W];
#pragma unroll
        for (int w = 0; w < W; ++w) far[w] = 0.0f;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) {
                const int64_t bi = (((int64_t)tzs[a] * L.qx + txs[bb]) * L.nd_up + 4 * (int64_t)ri.k) * kLB + l;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const float c4 =
                        up.get(bi, w) + up.get(bi + kLB, w) + up.get(bi + 2 * kLB, w) + up.get(bi + 3 * kLB, w);
                    far[w] = fmaf(wzs[a] * wxs[bb], 0.25f * c4, far[w]);
                }
            }
#pragma unroll
        for (int w = 0; w < W; ++w) I[w] = fmaf(T[w], far[w], I[w]);
    }
    if constexpr (W == 1) {
        epi.finish(ri, l, lane, I[0], op);
    } else {
        epi.finish_slots(ri, l, lane, I, op);
    }
}

// march_ray with the shared-direction walk (the 4 rows hold one direction).
template <class Op, class Epi, class Up>
__device__ __forceinline__ void march_ray_shared(const LevelDesc& L, int32_t nx, int32_t nz, Op& op, Epi& epi,
                                                 const double4* __restrict__ dirs, const Up& up, uint2* seg,
                                                 const RowCtx& cx_, int64_t ray, int32_t u, int32_t v, int32_t k,
                                                 bool active)
{
    RayInfo ri;
    ri.ray = ray;
    ri.active = active;
    ri.k = k;
    ri.u = u;
    ri.v = v;
    const double4 d = dirs[__builtin_amdgcn_readfirstlane(k)];
    ri.wx = d.x;
    ri.wz = d.y;
    op.begin_ray(d.x, d.y);
    constexpr int W = Op::kW;
    float I[W], T[W];
    walk_ray_shared(L, nx, nz, op, u, v, d, active, seg, cx_, I, T);
    merge_finish(L, op, epi, up, ri, cx_.l, cx_.lane, I, T);
}

// Probe and direction of launch-order ray r (of total): probe-major, or
// the tiled order of LevelDesc; active false past the end and on padding.
template <bool kShared = false>
__host__ __device__ __forceinline__ void ray_coords(const LevelDesc& L, int64_t r, int64_t total, int32_t& k,
                                                    int32_t& u, int32_t& v, bool& active)
{
    // 32-bit decode with the launch's divisors precomputed (set_decode
    // checks that its ray indices fit); a launch without them marches nothing
    const LevelDesc::Decode& D = L.dec;
    active = r < total && D.ready == kDecodeReady;
    const uint32_t rr = (uint32_t)(r < total ? r : total - 1);
    uint32_t kk, p;
    if (L.plist) {
        // sparse: entry i of the flagged-probe list stands for probe i of
        // the dense order (groups of tile_p^2 list entries when tiled)
        uint32_t i;
        if (L.tile_p <= 0) {
            i = D.nd.div(rr);
            kk = rr - i * D.nd.d;
        } else {
            const uint32_t g = D.per.div(rr), r_in = rr - g * D.per.d;
            const uint32_t t = D.nw.div(g), pl = D.tile_d.div(r_in);
            kk = (g - t * D.nw.d) * D.tile_d.d + (r_in - pl * D.tile_d.d);
            i = t * D.tp2.d + pl;
        }
        active = active && i < (uint32_t)L.n_active;
        p = (uint32_t)L.plist[i < (uint32_t)L.n_active ? i : L.n_active - 1];
        const uint32_t pv = D.px.div(p);
        u = (int32_t)(p - pv * D.px.d);
        v = (int32_t)pv;
        k = (int32_t)kk;
        return;
    }
    if (L.tile_p <= 0) {
        p = D.nd.div(rr);
        k = (int32_t)(rr - p * D.nd.d);
        const uint32_t pv = D.px.div(p);
        u = (int32_t)(p - pv * D.px.d);
        v = (int32_t)pv;
    } else {
        // group g = (probe tile, direction wedge), wedge fastest; within
        // a group, direction fastest (kShared: probe fastest)
        const uint32_t g = D.per.div(rr), r_in = rr - g * D.per.d;
        const uint32_t t = D.nw.div(g);
        uint32_t pl, kd;
        if (kShared) {
            kd = D.tp2.div(r_in);
            pl = r_in - kd * D.tp2.d;
        } else {
            pl = D.tile_d.div(r_in);
            kd = r_in - pl * D.tile_d.d;
        }
        k = (int32_t)((g - t * D.nw.d) * D.tile_d.d + kd);
        const uint32_t ty = D.ntx.div(t);
        uint32_t py = D.tile_p.div(pl), pxl = pl - py * D.tile_p.d;
        if (kShared) {
            // 4 consecutive probes (a wavefront's rows) run along the
            // direction's minor axis, where their clip ranges differ least:
            // theta_k = (2k + 1) pi / nd is x-major when (2k + 1) mod nd
            // lies within nd / 4 of 0 or nd
            const uint32_t m = 2u * (uint32_t)k + 1u, mm = m >= (uint32_t)L.nd ? m - (uint32_t)L.nd : m;
            const bool xmaj = 4u * mm <= (uint32_t)L.nd || 4u * mm >= 3u * (uint32_t)L.nd;
            if (xmaj) {
                const uint32_t tmp = py;
                py = pxl;
                pxl = tmp;
            }
        }
        u = (int32_t)((t - ty * D.ntx.d) * D.tile_p.d + pxl);
        v = (int32_t)(ty * D.tile_p.d + py);
        active = active && u < L.px && v < L.pz;
    }
    if (D.ready != kDecodeReady) k = u = v = 0;
}

// Waves per SIMD the march kernels are compiled for (their register
// budget): 4, except the one-batch bilinear fix, held to 5 (96 VGPRs; at
// the 99-102 it takes otherwise it runs 4 waves per SIMD and 10% slower).
// Holding the one-batch march to 7 spills and is slower than its 6.
template <class Op>
struct MarchWaves {
    static constexpr int rows = 4, fix = 4, shared = 4;
};
struct FieldOp;
template <>
struct MarchWaves<FieldOp> {
    static constexpr int rows = 4, fix = 5, shared = 4;
};

template <class Op, class Epi, class Up>
__global__ __launch_bounds__(kBlock, MarchWaves<Op>::rows) void k_march_rows(LevelDesc L, int32_t nx, int32_t nz, Op op, Epi epi,
                                                        const double4* __restrict__ dirs, Up up, int64_t total)
{
    // per wave, per row: (cell index, ds) entries, and staged step data
    __shared__ uint4 seg[kBlock / 64][4][kSegRow];
    __shared__ typename Op::Stage stg[Op::kStaged ? kBlock / 64 : 1][4][kStgRow];
    // block-wide tables of the Op (e.g. a line profile), copied once
    __shared__ float2 op_smem[Op::kSmemBytes > 0 ? Op::kSmemBytes / 8 : 2];
    if constexpr (Op::kSmemBytes > 0) {
        op.init_shared(op_smem);
        __syncthreads();
    }
    const RowCtx c = row_ctx();
    op.init(c.l);
    epi.init(c.l);
    up.init(c.l);
    {
        seg[c.w][c.row][c.l] = make_uint4(0u, 0u, 0u, 0u);
        if constexpr (Op::kStaged) {
            // positions past a row's segment count are read (with ds = 0):
            // they must hold zeros or a real record, never garbage
            static_assert(sizeof(typename Op::Stage) % 16 == 0, "stage entries are written as uint4");
            uint4* gw = reinterpret_cast<uint4*>(&stg[c.w][0][0]);
            constexpr int n16 = 4 * kStgRow * (int)sizeof(typename Op::Stage) / 16;
            for (int i = c.lane; i < n16; i += 64) gw[i] = make_uint4(0u, 0u, 0u, 0u);
        }
        wave_sync();
    }
    const unsigned lb = xcd_block_chunked(blockIdx.x, gridDim.x, L.dec);
    const int64_t stride = (int64_t)gridDim.x * kRaysPerBlock;
    for (int64_t base = ((int64_t)lb * (kBlock / 64) + c.w) * 4; base < total; base += stride) {
        int32_t k, u, v;
        bool active;
        ray_coords(L, base + c.row, total, k, u, v, active);
        const int64_t ray = ((int64_t)v * L.px + u) * L.nd + k;  // output index
        march_ray(L, nx, nz, op, epi, dirs, up, seg[c.w], stg[Op::kStaged ? c.w : 0], c, ray, u, v, k, active);
    }
}

// The march with the shared-direction walk, for tiled launch orders with an
// even tile_p and an integral probe spacing: the rays of a tile run probe
// fastest (ray_coords<true>), so the 4 rows of every wavefront are 4 probes
// of one direction (total is a multiple of 4: whole tiles).
template <class Op, class Epi, class Up>
__global__ __launch_bounds__(kBlock, MarchWaves<Op>::shared) void k_march_shared(LevelDesc L, int32_t nx, int32_t nz, Op op,
                                                                             Epi epi, const double4* __restrict__ dirs,
                                                                             Up up, int64_t total)
{
    __shared__ uint2 seg[kBlock / 64][kSegShared];
    const RowCtx c = row_ctx();
    op.init(c.l);
    epi.init(c.l);
    up.init(c.l);
    const unsigned lb = xcd_block_chunked(blockIdx.x, gridDim.x, L.dec);
    const int64_t stride = (int64_t)gridDim.x * kRaysPerBlock;
    for (int64_t base = ((int64_t)lb * (kBlock / 64) + c.w) * 4; base < total; base += stride) {
        int32_t k, u, v;
        bool active;
        ray_coords<true>(L, base + c.row, total, k, u, v, active);
        const int64_t ray = ((int64_t)v * L.px + u) * L.nd + k;  // output index
        march_ray_shared(L, nx, nz, op, epi, dirs, up, seg[c.w], c, ray, u, v, k, active);
    }
}

// Bilinear fix (Sec. 2.5): the interval (u, v, k) of a cascade below the
// top is traced once per bilinear probe q of the cascade above, from its
// usual start p + t_a w_k to the start q + t_b w_k of the child cone on q
// (the cone of k's four children, centred on w_k), merged with q's children
// 4k..4k+3, and the four results are summed with the bilinear weights. The
// 4 rows of a wavefront are the 4 taps of one interval (row = 2 * a + b for
// tap z index a, x index b), so the sum is two cross-row shuffles; row 0
// finishes the interval. With Op::kW = 2 each lane carries two wavelength
// batches along the same four walks. Taps are clamped at the grid edge (as in the
// basic merge) and keep their weights.
template <class Op, class Epi, class Up>
__device__ __forceinline__ void march_fix_ray(const LevelDesc& L, int32_t nx, int32_t nz, Op& op, Epi& epi,
                                              const double4* __restrict__ dirs, const Up& up, uint4 (*seg)[kSegRow],
                                              typename Op::Stage (*stg)[kStgRow], const RowCtx& cx_, int64_t ray,
                                              int32_t u, int32_t v, int32_t k, bool active)
{
    constexpr int W = Op::kW;  // wavelength batches per lane
    const int row = cx_.row, l = cx_.l;
    const int ta_z = row >> 1, ta_x = row & 1;
    // the same taps and weights as the basic merge
    const int bx0 = (u - 1) >> 1, bz0 = (v - 1) >> 1;
    const float fx = (u & 1) ? 0.25f : 0.75f;
    const float fz = (v & 1) ? 0.25f : 0.75f;
    const int tx = min(max(bx0 + ta_x, 0), L.qx - 1);
    const int tz = min(max(bz0 + ta_z, 0), L.qz - 1);
    const float wgt = (ta_x ? fx : 1.0f - fx) * (ta_z ? fz : 1.0f - fz);

    const double4 dk = dirs[k];
    const double s_up = 2.0 * L.s;
    const double ax = (u + 0.5) * L.s + L.ta * dk.x, az = (v + 0.5) * L.s + L.ta * dk.y;
    const double ex = (tx + 0.5) * s_up + L.tb * dk.x, ez = (tz + 0.5) * s_up + L.tb * dk.y;
    const double dx = ex - ax, dz = ez - az;
    const double len = sqrt(dx * dx + dz * dz);
    // a zero-length ray walks nothing (any unit direction will do); an
    // axis-parallel one gets a 1e-12 minor component, so its plane steps on
    // that axis stay finite (its cells are unchanged)
    double4 d = make_double4(0.6, 0.8, 1.0 / 0.6, 1.0 / 0.8);
    if (len > 0.0) {
        double wx = dx / len, wz = dz / len;
        if (fabs(wx) < 1e-12) wx = wx < 0.0 ? -1e-12 : 1e-12;
        if (fabs(wz) < 1e-12) wz = wz < 0.0 ? -1e-12 : 1e-12;
        d = make_double4(wx, wz, 1.0 / wx, 1.0 / wz);
    }
    op.begin_ray(dk.x, dk.y);
    float I[W], T[W];
    walk_ray(L, nx, nz, op, ax, az, d, 0.0, len, active && len > 0.0, seg, stg, cx_, I, T);

    if (active && L.has_up) {
        const int64_t bi = (((int64_t)tz * L.qx + tx) * L.nd_up + 4 * (int64_t)k) * kLB + l;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const float c4 = up.get(bi, w) + up.get(bi + kLB, w) + up.get(bi + 2 * kLB, w) + up.get(bi + 3 * kLB, w);
            I[w] = fmaf(T[w], 0.25f * c4, I[w]);
        }
    }
    float sum[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        sum[w] = wgt * I[w];
        sum[w] += __shfl_xor(sum[w], 16);
        sum[w] += __shfl_xor(sum[w], 32);
    }
    RayInfo ri;
    ri.ray = ray;
    ri.active = active && row == 0;
    ri.k = k;
    ri.u = u;
    ri.v = v;
    ri.wx = dk.x;
    ri.wz = dk.y;
    if constexpr (W == 1) {
        epi.finish(ri, l, cx_.lane, sum[0], op);
    } else {
        epi.finish_slots(ri, l, cx_.lane, sum, op);
    }
}

// One interval per wavefront (its 4 taps on the 4 rows); total = intervals
// of the launch (the tiled order of LevelDesc applies to intervals).
template <class Op, class Epi, class Up>
__global__ __launch_bounds__(kBlock, MarchWaves<Op>::fix) void k_march_fix(LevelDesc L, int32_t nx, int32_t nz, Op op, Epi epi,
                                                       const double4* __restrict__ dirs, Up up, int64_t total)
{
    static_assert(!Op::kStaged && Op::kSmemBytes == 0, "the fix takes per-lane field ops");
    __shared__ uint4 seg[kBlock / 64][4][kSegRow];
    __shared__ typename Op::Stage stg[1][4][kStgRow];
    const RowCtx c = row_ctx();
    op.init(c.l);
    epi.init(c.l);
    up.init(c.l);
    seg[c.w][c.row][c.l] = make_uint4(0u, 0u, 0u, 0u);
    wave_sync();
    const unsigned lb = xcd_block_chunked(blockIdx.x, gridDim.x, L.dec);
    const int64_t stride = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t r = (int64_t)lb * (kBlock / 64) + c.w; r < total; r += stride) {
        int32_t k, u, v;
        bool active;
        ray_coords(L, r, total, k, u, v, active);
        const int64_t ray = ((int64_t)v * L.px + u) * L.nd + k;
        march_fix_ray(L, nx, nz, op, epi, dirs, up, seg[c.w], stg[0], c, ray, u, v, k, active);
    }
}

// Epilogue that stores the merged radiance of every ray: out[ray][16].
struct StoreEpi {
    float* out;
    __device__ __forceinline__ void init(int) {}
    template <class Op>
    __device__ __forceinline__ void finish(const RayInfo& ri, int l, int lane, float I, const Op&)
    {
        (void)lane;
        if (ri.active) out[ri.ray * kLB + l] = I;
    }
};

// Epilogue storing the 16-bit codes with the wavelength's exponent bias
// (enc_h16; no merged radiance exceeds the largest source function of its
// wavelength, which sets the bias).
struct StoreF16Epi {
    uint16_t* out;
    const int32_t* ebias_b;  // [16] of this batch
    int32_t B = 0;
    __device__ __forceinline__ void init(int l) { B = ebias_b[l] * 1024; }
    template <class Op>
    __device__ __forceinline__ void finish(const RayInfo& ri, int l, int lane, float I, const Op&)
    {
        (void)lane;
        if (ri.active) out[ri.ray * kLB + l] = enc_h16(I, B);
    }
};

// Cascade-0 epilogue writing J directly: with N_0 = 4 directions the 4 rows
// of a wavefront are the 4 directions of one cell (ray = cell * 4 + k), so
// J = (1/4) sum over the rows, J[lam0 + l][cell] for l < n_valid.
// With an inclination quadrature, pass m writes w_m J_m (acc false) or adds
// it (acc true); flatland: w = 1, acc false.
struct JEpi {
    float* J;
    int32_t lam0, n_valid;
    int64_t ncell;
    float w = 1.0f;
    bool acc = false;
    __device__ __forceinline__ void init(int) {}
    template <class Op>
    __device__ __forceinline__ void finish(const RayInfo& ri, int l, int lane, float I, const Op&)
    {
        float s = I + __shfl_xor(I, 16);
        s += __shfl_xor(s, 32);
        if (ri.active && (lane >> 4) == 0 && l < n_valid) {
            float* j = &J[(int64_t)(lam0 + l) * ncell + ri.ray / 4];
            const float v = (0.25f * w) * s;
            if (acc)
                *j += v;
            else
                *j = v;
        }
    }
};

// Opacity from a per-batch field F[c][16] = {optical depth per cell in log2
// units, S}, read with buffer loads: an out-of-range offset returns 0.
struct FieldOp {
    const float2* Fb;
    uint32_t fb_bytes;
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t lane_off;
    using Raw = float2;
    static constexpr int kW = 1;
    static constexpr bool kStaged = false;  // per-lane data: nothing to stage
    struct Stage {};
    struct StageIn {};
    static constexpr int kSmemBytes = 0;
    __device__ __forceinline__ void init_shared(float2*) {}
    __device__ __forceinline__ void init(int l)
    {
        rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)Fb, 0, (int)fb_bytes, 0x00020000);
        lane_off = (uint32_t)l * 8u;
    }
    __device__ __forceinline__ void begin_ray(double, double) {}
    // key of a cell: the byte offset of its 16 wavelengths, cell * 128 B
    // (cell < 2^24, so at most 2^31 - 128, and key + lane offset < 2^31);
    // the null key 2^31 lies at or beyond every buffer's size and reads zeros
    static constexpr uint32_t kNullKey = 0x80000000u;
    __device__ __forceinline__ uint32_t key(uint32_t cell) const { return cell * (uint32_t)(kLB * 8); }
    __device__ __forceinline__ void fetch_key(uint32_t k, Raw (&r)[kW]) const
    {
        r[0] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rsrc, k + lane_off, 0, 0));
    }
    __device__ __forceinline__ float2 resolve(const Raw& r) const { return r; }
};

// Two consecutive batches of the same field layout per lane (Fb and
// Fb + ncell * 16): one segment list, one key, two buffer loads.
struct FieldOp2 {
    const float2* Fb;
    uint32_t fb_bytes;  // bytes of one batch
    __amdgpu_buffer_rsrc_t rsrc0, rsrc1;
    uint32_t lane_off;
    using Raw = float2;
    static constexpr int kW = 2;
    static constexpr bool kStaged = false;
    struct Stage {};
    struct StageIn {};
    static constexpr int kSmemBytes = 0;
    __device__ __forceinline__ void init_shared(float2*) {}
    __device__ __forceinline__ void init(int l)
    {
        rsrc0 = __builtin_amdgcn_make_buffer_rsrc((void*)Fb, 0, (int)fb_bytes, 0x00020000);
        rsrc1 = __builtin_amdgcn_make_buffer_rsrc((void*)((const char*)Fb + fb_bytes), 0, (int)fb_bytes, 0x00020000);
        lane_off = (uint32_t)l * 8u;
    }
    __device__ __forceinline__ void begin_ray(double, double) {}
    static constexpr uint32_t kNullKey = 0x80000000u;
    __device__ __forceinline__ uint32_t key(uint32_t cell) const { return cell * (uint32_t)(kLB * 8); }
    __device__ __forceinline__ void fetch_key(uint32_t k, Raw (&r)[kW]) const
    {
        r[0] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rsrc0, k + lane_off, 0, 0));
        r[1] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rsrc1, k + lane_off, 0, 0));
    }
    __device__ __forceinline__ float2 resolve(const Raw& r) const { return r; }
};

// Epilogues for two batches per lane: slot 1 is stored `stride` elements
// after slot 0 (16-bit codes with the next batch's biases).
struct StoreEpi2 {
    float* out;
    int64_t stride;
    __device__ __forceinline__ void init(int) {}
    template <class Op>
    __device__ __forceinline__ void finish_slots(const RayInfo& ri, int l, int, const float (&I)[2], const Op&)
    {
        if (ri.active) {
            out[ri.ray * kLB + l] = I[0];
            out[stride + ri.ray * kLB + l] = I[1];
        }
    }
};
struct StoreF16Epi2 {
    uint16_t* out;
    int64_t stride;
    const int32_t* ebias_b;  // [32]: this batch's biases, then the next batch's
    int32_t B0 = 0, B1 = 0;
    __device__ __forceinline__ void init(int l)
    {
        B0 = ebias_b[l] * 1024;
        B1 = ebias_b[l + kLB] * 1024;
    }
    template <class Op>
    __device__ __forceinline__ void finish_slots(const RayInfo& ri, int l, int, const float (&I)[2], const Op&)
    {
        if (ri.active) {
            out[ri.ray * kLB + l] = enc_h16(I[0], B0);
            out[stride + ri.ray * kLB + l] = enc_h16(I[1], B1);
        }
    }
};
// Cascade 0 with N_0 = 4: J of both batches (rows lam0 + l and
// lam0 + 16 + l, for l below each batch's valid count).
struct JEpi2 {
    float* J;
    int32_t lam0, n_valid0, n_valid1;
    int64_t ncell;
    float w = 1.0f;
    bool acc = false;
    __device__ __forceinline__ void init(int) {}
    template <class Op>
    __device__ __forceinline__ void finish_slots(const RayInfo& ri, int l, int lane, const float (&I)[2], const Op&)
    {
        float s0 = I[0] + __shfl_xor(I[0], 16);
        float s1 = I[1] + __shfl_xor(I[1], 16);
        s0 += __shfl_xor(s0, 32);
        s1 += __shfl_xor(s1, 32);
        if (ri.active && (lane >> 4) == 0) {
            const float q = 0.25f * w;
            float* j0 = &J[(int64_t)(lam0 + l) * ncell + ri.ray / 4];
            float* j1 = &J[(int64_t)(lam0 + kLB + l) * ncell + ri.ray / 4];
            if (acc) {
                if (l < n_valid0) *j0 += q * s0;
                if (l < n_valid1) *j1 += q * s1;
            } else {
                if (l < n_valid0) *j0 = q * s0;
                if (l < n_valid1) *j1 = q * s1;
            }
        }
    }
};


// W inclination rays per lane (2D invariance): the rays of one wavelength
// batch with the same x-z projection, inclined to the invariant y axis. One
// field load per step serves all W; slot w scales the optical depth by its
// path per projected cell, sc[w] = 1 / sin(inclination).
template <int W>
struct FieldOpIncl {
    const float2* Fb;
    uint32_t fb_bytes;
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t lane_off;
    float sc[W];
    using Raw = float2;
    static constexpr int kW = W;
    static constexpr bool kStaged = false;
    struct Stage {};
    struct StageIn {};
    static constexpr int kSmemBytes = 0;
    __device__ __forceinline__ void init_shared(float2*) {}
    __device__ __forceinline__ void init(int l)
    {
        rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)Fb, 0, (int)fb_bytes, 0x00020000);
        lane_off = (uint32_t)l * 8u;
    }
    __device__ __forceinline__ void begin_ray(double, double) {}
    static constexpr uint32_t kNullKey = 0x80000000u;
    __device__ __forceinline__ uint32_t key(uint32_t cell) const { return cell * (uint32_t)(kLB * 8); }
    __device__ __forceinline__ void fetch_key(uint32_t k, Raw (&r)[kW]) const
    {
        const float2 f = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rsrc, k + lane_off, 0, 0));
#pragma unroll
        for (int w = 0; w < W; ++w) r[w] = make_float2(f.x * sc[w], f.y);
    }
    __device__ __forceinline__ float2 resolve(const Raw& r) const { return r; }
};

// Inclination slots stored `stride` elements apart.
template <int W>
struct StoreEpiSlots {
    float* out;
    int64_t stride;
    __device__ __forceinline__ void init(int) {}
    template <class Op>
    __device__ __forceinline__ void finish_slots(const RayInfo& ri, int l, int, const float (&I)[W], const Op&)
    {
        if (ri.active) {
#pragma unroll
            for (int w = 0; w < W; ++w) out[w * stride + ri.ray * kLB + l] = I[w];
        }
    }
};

// 16-bit codes of W slots `stride` elements apart, slot w with the biases
// of batch b + w (ebias_b[w * 16 + l]).
template <int W>
struct StoreF16EpiSlots {
    uint16_t* out;
    int64_t stride;
    const int32_t* ebias_b;  // [W][16]
    __device__ __forceinline__ void init(int) {}
    template <class Op>
    __device__ __forceinline__ void finish_slots(const RayInfo& ri, int l, int, const float (&I)[W], const Op&)
    {
        if (ri.active) {
#pragma unroll
            for (int w = 0; w < W; ++w)
                out[w * stride + ri.ray * kLB + l] = enc_h16(I[w], ebias_b[l + w * kLB] * 1024);
        }
    }
};

// Cascade 0 with N_0 = 4 and W inclination slots: J = (1/4) sum over the
// rows of sum_w wt[w] I_w (the quadrature weights sum to 1).
template <int W>
struct JEpiIncl {
    float* J;
    int32_t lam0, n_valid;
    int64_t ncell;
    float wt[W];
    __device__ __forceinline__ void init(int) {}
    template <class Op>
    __device__ __forceinline__ void finish_slots(const RayInfo& ri, int l, int lane, const float (&I)[W], const Op&)
    {
        float v = 0.0f;
#pragma unroll
        for (int w = 0; w < W; ++w) v = fmaf(wt[w], I[w], v);
        float s = v + __shfl_xor(v, 16);
        s += __shfl_xor(s, 32);
        if (ri.active && (lane >> 4) == 0 && l < n_valid) J[(int64_t)(lam0 + l) * ncell + ri.ray / 4] = 0.25f * s;
    }
};

}  // namespace march
}  // namespace rcx
