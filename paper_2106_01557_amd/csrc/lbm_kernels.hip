// HIP kernels for gfx950 (MI355X): the lattice update of the liquid-vapour
// double-distribution model and its diagnostics.
//
// Layout in HBM: row-interleaved structure of arrays [y][s][x]: for each lattice row
// y, the 18 population rows (slot s < 9 is f_s, slot 9 + s is g_s) follow each other,
// x fastest.  A wavefront's 36 row accesses of one step then fall in three
// contiguous blocks of 18 rows instead of 18 planes far apart, which keeps the DRAM
// page and channel pattern close to a plain copy.
// Velocity order (SM Eq. (1)): 0 rest, 1 (+x), 2 (+y), 3 (-x), 4 (-y),
// 5 (+x,+y), 6 (-x,+y), 7 (-x,-y), 8 (+x,-y).
//
// The per-node arithmetic follows the paper's moment-space form: M of SM Eq. (2)
// applied as sums and differences, the equilibria and sources of SM Eqs. (3)-(4),
// the collision matrices S and L of SM Eq. (5) (only their non-trivial rows),
// the compensation Q_m and dissipation Y of SM Eq. (6), the moments of Eq. (14)
// and the closure p_LBE = c_s^2 (rho + eta) = p_BE (Eq. (15)).  No MFMA: the
// update is not a contraction; it is bound by HBM traffic (36 values per node
// per step in the fused two-buffer scheme).

#include <cstdlib>

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lbm_internal.hpp"
#include "lbm_model.hpp"

namespace lbm_dev {
namespace {

// ---------------------------------------------------------------------------
// storage <-> arithmetic conversions; 16-bit formats store deviations from a
// per-population reference (the rest equilibrium of a reference state)
// ---------------------------------------------------------------------------
template <typename S, typename C>
struct Io;

template <>
struct Io<double, double> {
    __device__ static double ld(const double* p, int k, double) { return p[k]; }
    __device__ static void st(double* p, int k, double v, double) { p[k] = v; }
};
template <>
struct Io<float, float> {
    __device__ static float ld(const float* p, int k, float) { return p[k]; }
    __device__ static void st(float* p, int k, float v, float) { p[k] = v; }
};
// FP16 deviation v - ref, rounded once from the exact difference to FP16 (the
// mixed-precision FMA v * 1 + (-ref) with an FP16 result).  Every FP16 store of the
// library goes through this conversion or its pair form below, so all kernel forms
// round alike.
__device__ inline unsigned short f16_dev(float v, float ref) {
    unsigned t;
    asm("v_fma_mixlo_f16 %0, %1, 1.0, -%2" : "=v"(t) : "v"(v), "v"(ref));
    return (unsigned short)(t & 0xffffu);
}
template <>
struct Io<__half, float> {
    __device__ static float ld(const __half* p, int k, float ref) { return __half2float(p[k]) + ref; }
    __device__ static void st(__half* p, int k, float v, float ref) {
        p[k] = __builtin_bit_cast(__half, f16_dev(v, ref));
    }
};
template <>
struct Io<__hip_bfloat16, float> {
    __device__ static float ld(const __hip_bfloat16* p, int k, float ref) {
        return __bfloat162float(p[k]) + ref;
    }
    __device__ static void st(__hip_bfloat16* p, int k, float v, float ref) {
        p[k] = __float2bfloat16(v - ref);
    }
};

// ---------------------------------------------------------------------------
// stochastic rounding of the 16-bit stores (lbm_params.rounding)
// ---------------------------------------------------------------------------
// gfx950's v_cvt_sr_f16_f32 / v_cvt_sr_bf16_f32 add the top 13 (FP16) or 16 (BF16) bits
// of a 32-bit random word below the kept mantissa bits and truncate, so a value rounds
// away from zero with probability equal to its discarded fraction (checked on the GPU
// over all 2^16 high-half words for values of both signs, normal and subnormal).  The
// random word of a stored value is h ^ salt: h hashes the step count and the node (the
// byte offset of the node's column pair within the state, which is the same in every
// kernel form and in batches), and the salt separates the 18 slots and the two columns
// of a pair.  The hash is a multiply-xorshift finalizer (the constants of C. Wellons'
// "lowbias32").
__host__ __device__ constexpr uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
struct SaltTable {
    uint32_t v[36];  // [column parity * 18 + slot]
};
constexpr SaltTable make_salts() {
    SaltTable t{};
    for (uint32_t k = 0; k < 36; ++k) t.v[k] = mix32((k + 1u) * 0x9E3779B9u);
    return t;
}
__device__ constexpr SaltTable kSrSalt = make_salts();

__device__ inline uint32_t sr_key(uint32_t step) { return mix32(step * 0x9E3779B9u + 0x632BE5ABu); }

// hash of the column pair at byte offset o under the step key
template <typename Off>
__device__ inline uint32_t sr_node(Off o, uint32_t key) {
    uint32_t lo = (uint32_t)o;
    if constexpr (sizeof(Off) > 4) lo ^= (uint32_t)((uint64_t)o >> 32);
    return mix32(lo ^ key);
}

// deviation v - ref stochastically rounded; pairs put the first column in the low half
template <typename S>
struct Sr16;
template <>
struct Sr16<__half> {
    using V2 = _Float16 __attribute__((ext_vector_type(2)));
    __device__ static unsigned pack(float a, float b, float ref, uint32_t ra, uint32_t rb) {
        V2 t = {};
        t = __builtin_amdgcn_cvt_sr_f16_f32(t, a - ref, ra, false);
        t = __builtin_amdgcn_cvt_sr_f16_f32(t, b - ref, rb, true);
        return __builtin_bit_cast(unsigned, t);
    }
    __device__ static unsigned short one(float v, float ref, uint32_t r) {
        V2 t = {};
        t = __builtin_amdgcn_cvt_sr_f16_f32(t, v - ref, r, false);
        return (unsigned short)(__builtin_bit_cast(unsigned, t) & 0xffffu);
    }
};
template <>
struct Sr16<__hip_bfloat16> {
    using V2 = __bf16 __attribute__((ext_vector_type(2)));
    __device__ static unsigned pack(float a, float b, float ref, uint32_t ra, uint32_t rb) {
        V2 t = {};
        t = __builtin_amdgcn_cvt_sr_bf16_f32(t, a - ref, ra, false);
        t = __builtin_amdgcn_cvt_sr_bf16_f32(t, b - ref, rb, true);
        return __builtin_bit_cast(unsigned, t);
    }
    __device__ static unsigned short one(float v, float ref, uint32_t r) {
        V2 t = {};
        t = __builtin_amdgcn_cvt_sr_bf16_f32(t, v - ref, r, false);
        return (unsigned short)(__builtin_bit_cast(unsigned, t) & 0xffffu);
    }
};

// ---------------------------------------------------------------------------
// fused two-buffer step (pull streaming, aligned strips)
// ---------------------------------------------------------------------------
// State convention of the two-buffer scheme: a buffer holds the post-collision
// populations at the node where they were computed, not yet streamed; step t
// reads f_i(x, t) = f_bar_i(x - e_i, t - dt) (Eq. (12a) applied on read) and
// writes f_bar(x, t) at x.
//
// A wavefront owns an aligned strip of 64 columns (one per lane; k_step_ab) or 128
// columns (two adjacent columns per lane; k_step_ab2) and marches through `rows`
// rows.  For the populations of target row y it loads, for each i, the aligned row
// y - e_iy of slot i (one contiguous segment per instruction) and moves the values
// e_ix columns across lanes with a wave-wide DPP shift.  The one value per shifted
// population that comes from outside the strip (for lane 0 or the last owned lane)
// and the populations of the two halo columns (whose densities the force stencil
// needs) arrive through one gather load per row in which each of 18 lanes fetches
// one value.  Stores are aligned, at the node.  Densities of the rows y-1, y, y+1
// live in registers; their x-neighbours come from DPP shifts as well.  Every
// population is read from HBM once per step.


// Wave-wide one-lane shifts.  The lane with no source (0 for west, 63 for east) reads
// zero (bound_ctrl); callers replace that lane's value with a gathered one.
__device__ inline float dpp_from_west(float v) {  // lane L receives lane L-1
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
__device__ inline float dpp_from_east(float v) {  // lane L receives lane L+1
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}
__device__ inline double dpp_from_west(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x138, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double dpp_from_east(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), 0x130, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x130, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ inline float lane_value(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ inline double lane_value(double v, int l) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Index modulo n (for uniform values; the division only runs when v is outside [0, n)).
__device__ inline int wrap_row(int v, int n) {
    if (v < 0 || v >= n) v = ((v % n) + n) % n;
    return v;
}

// Addressing: with kBuf every access is a raw buffer instruction on one resource
// per state buffer whose record count covers the whole buffer; for row accesses the
// slot offset (s times the bytes of one population row) goes in the scalar offset and
// the lane's row-block/column byte offset in the vector offset, for the gather the
// whole offset is per lane.  A lane that must not store, or whose gather slot is
// unused, gets the vector offset drop = (2^32 - 16 - 17 * row_bytes) rounded down to
// a multiple of 16: for every slot every dword of an access of up to 16 bytes then
// lies at or past the record count and below 2^32, so the hardware drops the store
// (or returns zero) whether or not it counts the scalar offset in its range check,
// and no component offset wraps around.  That needs buffer_bytes + 17 * row_bytes +
// 32 < 2^32 (checked by fits_32bit); larger lattices use 64-bit addresses and
// branches instead.
//
// Stores carry the non-temporal cache policy: a step writes every byte of the output
// state once and no kernel of the same step reads it again, so the stores should not
// displace the input lines that the neighbouring strips' halo gathers still reuse.
constexpr int kStreamStore = 2;  // cache-policy operand of the buffer stores: nt

template <typename S>
struct Bits;
template <>
struct Bits<float> {
    __device__ static float ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
    }
    __device__ static void st(float x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, kStreamStore);
    }
};
template <>
struct Bits<double> {
    using V2 = unsigned __attribute__((ext_vector_type(2)));
    __device__ static double ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
    }
    __device__ static void st(double x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, x), r, v, s, kStreamStore);
    }
};
template <>
struct Bits<__half> {
    __device__ static __half ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return __builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
    }
    __device__ static void st(__half x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, kStreamStore);
    }
};
template <>
struct Bits<__hip_bfloat16> {
    __device__ static __hip_bfloat16 ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return __builtin_bit_cast(__hip_bfloat16, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
    }
    __device__ static void st(__hip_bfloat16 x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, kStreamStore);
    }
};

template <typename S, bool kBuf>
struct Planes;

// Byte offsets within a state buffer: 32 bits on the buffer-instruction path.
template <bool kBuf>
struct OffT {
    using type = size_t;
};
template <>
struct OffT<true> {
    using type = unsigned;
};

template <typename S>
struct Planes<S, true> {
    __amdgpu_buffer_rsrc_t r;
    unsigned ps, drop;  // ps: bytes of one population row (the slot stride)
    __device__ Planes(const void* base, size_t total_bytes, unsigned row_bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)(unsigned)total_bytes, 0x00020000)),
          ps(row_bytes),
          drop((0xFFFFFFF0u - 17u * row_bytes) & ~15u) {}
    template <typename C>
    __device__ C ld(int i, unsigned off, C ref) const {
        const S v = Bits<S>::ld(r, off, ps * (unsigned)i);
        return Io<S, C>::ld(&v, 0, ref);
    }
    // per-lane slot; an unused gather slot reads zero
    template <typename C>
    __device__ C gather(unsigned slot, unsigned off, bool on, C ref) const {
        const S v = Bits<S>::ld(r, on ? ps * slot + off : drop, 0u);
        return Io<S, C>::ld(&v, 0, ref);
    }
    // 16-bit storage: the gathered bits, converted later (unpack_gather)
    template <typename C>
    __device__ C gather_raw(unsigned slot, unsigned off, bool on) const {
        const S v = Bits<S>::ld(r, on ? ps * slot + off : drop, 0u);
        return __builtin_bit_cast(C, (unsigned)__builtin_bit_cast(unsigned short, v));
    }
    template <typename C>
    __device__ void st(int i, unsigned off, C v, C ref, bool valid) const {
        S t;
        Io<S, C>::st(&t, 0, v, ref);
        Bits<S>::st(t, r, valid ? off : drop, ps * (unsigned)i);
    }
    // 16-bit storage, stochastic rounding with the random word rnd
    template <typename C>
    __device__ void st_sr(int i, unsigned off, C v, C ref, uint32_t rnd, bool valid) const {
        Bits<S>::st(__builtin_bit_cast(S, Sr16<S>::one(v, ref, rnd)), r, valid ? off : drop, ps * (unsigned)i);
    }
};

// Non-temporal store of one value through a plain pointer (64-bit address path).
template <typename S, typename C>
__device__ inline void stream_store(S* p, C v, C ref) {
    S t;
    Io<S, C>::st(&t, 0, v, ref);
    if constexpr (sizeof(S) == 8)
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned long long, t), reinterpret_cast<unsigned long long*>(p));
    else if constexpr (sizeof(S) == 4)
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned, t), reinterpret_cast<unsigned*>(p));
    else
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, t), reinterpret_cast<unsigned short*>(p));
}

template <typename S>
struct Planes<S, false> {
    char* base;
    size_t ps;
    __device__ Planes(const void* b, size_t, unsigned row_bytes) : base((char*)b), ps(row_bytes) {}
    template <typename C>
    __device__ C ld(int i, size_t off, C ref) const {
        return Io<S, C>::ld(reinterpret_cast<const S*>(base + ps * i + off), 0, ref);
    }
    template <typename C>
    __device__ C gather(unsigned slot, size_t off, bool on, C ref) const {
        // unused slots read slot 0 at offset 0 (a valid address) and are ignored
        return on ? Io<S, C>::ld(reinterpret_cast<const S*>(base + ps * slot + off), 0, ref) : C(0);
    }
    template <typename C>
    __device__ C gather_raw(unsigned slot, size_t off, bool on) const {
        const S v = *reinterpret_cast<const S*>(base + ps * slot + off);
        return on ? __builtin_bit_cast(C, (unsigned)__builtin_bit_cast(unsigned short, v)) : C(0);
    }
    template <typename C>
    __device__ void st(int i, size_t off, C v, C ref, bool valid) const {
        if (valid) stream_store(reinterpret_cast<S*>(base + ps * i + off), v, ref);
    }
    template <typename C>
    __device__ void st_sr(int i, size_t off, C v, C ref, uint32_t rnd, bool valid) const {
        if (valid)
            __builtin_nontemporal_store(Sr16<S>::one(v, ref, rnd),
                                        reinterpret_cast<unsigned short*>(base + ps * i + off));
    }
};

template <typename C>
__device__ inline C sum9(const C* f) {
    return f[0] + ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
}

// Geometry of one strip, per lane.  The gather slot of a lane (18 for f, 6 for g)
// names a population, a column and the row offset -e_y of that population.
struct Strip {
    int nx, ny;
    unsigned rowb, esz;   // bytes of one population row; bytes per value
    unsigned xc;          // the lane's column (clamped to a valid column past the strip end)
    bool owner;           // the lane holds an owned column
    int last;             // last owned lane
    // gather slots
    bool fon, gon;
    unsigned fplane, gplane, fcol, gcol;
    int fdy, gdy;
    float fref, gref;  // 16-bit storage: deviation references of the gather slots' populations
    uint32_t srkey;    // stochastic rounding: key of this step's random stream
};

// ref[k] for a per-lane k in [0, 9) by selects (no indexed memory access)
template <typename C>
__device__ inline C pick9(const C* ref, unsigned k) {
    C r = ref[0];
#pragma unroll
    for (unsigned i = 1; i < 9; ++i) r = k == i ? ref[i] : r;
    return r;
}

// Raw loads for one target row: slot i at source row y - e_iy, aligned, and the
// gather.  up/mid/dn are the byte offsets of the row blocks of source rows y+1, y,
// y-1 (periodic).
template <typename S, typename C, bool kBuf>
__device__ inline void load_target_row(const Planes<S, kBuf>& B, int first, const Strip& G,
                                       typename OffT<kBuf>::type up, typename OffT<kBuf>::type mid,
                                       typename OffT<kBuf>::type dn, bool is_f, const C* ref, C* raw, C& gth) {
    using Off = typename OffT<kBuf>::type;
    const unsigned xo = G.xc * G.esz;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const Off r = kEy[i] < 0 ? up : (kEy[i] > 0 ? dn : mid);
        raw[i] = B.template ld<C>(first + i, r + xo, ref[i]);
    }
    const unsigned plane = is_f ? G.fplane : G.gplane;
    const unsigned col = is_f ? G.fcol : G.gcol;
    const int dy = is_f ? G.fdy : G.gdy;  // -e_y of the slot's population
    const bool on = is_f ? G.fon : G.gon;
    const Off r = dy > 0 ? up : (dy < 0 ? dn : mid);
    // the gather's reference is the slot's own (it differs per lane)
    gth = B.template gather<C>(first + plane, r + col * G.esz, on, ref[plane]);
}

// Byte offset of the next row block, periodic in y: one conditional subtraction is
// exact because the offset is always below the buffer size.
template <typename Off>
__device__ inline Off next_row(Off o, Off block, Off total) {
    o += block;
    return o >= total ? o - total : o;
}

// Streamed populations of the target row from its raw loads (DPP shifts plus the
// edge values from the gather) and the densities of the row's lanes and of its two
// halo columns.  Gather slots for f: 0-2 pops 0,2,4 at x0-1; 3-5 pops 1,5,8 at x0-2;
// 6-8 pops 1,5,8 at x0-1; 9-11 pops 0,2,4 at x0+n; 12-14 pops 3,6,7 at x0+n+1;
// 15-17 pops 3,6,7 at x0+n (n = owned columns).  For g: 0-2 pops 1,5,8 at x0-1;
// 3-5 pops 3,6,7 at x0+n.
// DPP reads a source lane only if that lane is active, so every shift below runs
// with the whole wavefront active: shifts and lane reads are computed unconditionally
// and pinned (empty asm) before the per-lane selects, which the compiler must not
// turn into branches around the shifts.
template <typename C>
__device__ inline void pin(C& v) {
    asm volatile("" : "+v"(v));
}

// A copy of a landed load into a register of its own (early clobber: never the source's).
// Without it the register allocator lets a population that passes straight from a raw
// load into the row arrays share the load's register, and the next load of that array
// then has to go elsewhere, which costs a rotation of copies of in-flight loads at the
// loop's back edge (each such copy waits for its load).
__device__ inline float fresh(float v) {
    float t;
    asm("v_mov_b32 %0, %1" : "=&v"(t) : "v"(v));
    return t;
}
__device__ inline double fresh(double v) {
    double t;
    asm("v_mov_b64 %0, %1" : "=&v"(t) : "v"(v));
    return t;
}
// 16-bit storage converts every loaded value, which already gives it a register of
// its own: the copy is needed only where raw loads feed the arrays directly.
template <bool kCopy, typename C>
__device__ inline C pass(C v) {
    if constexpr (kCopy)
        return fresh(v);
    else
        return v;
}

template <bool kCopy, typename C>
__device__ inline void finish_f(const Strip& G, const C* raw, C gth, C* f, C& rho, C& rhoL, C& rhoR) {
    const int lane = threadIdx.x & 63;
    C w1 = dpp_from_west(raw[1]), w5 = dpp_from_west(raw[5]), w8 = dpp_from_west(raw[8]);
    C e3 = dpp_from_east(raw[3]), e6 = dpp_from_east(raw[6]), e7 = dpp_from_east(raw[7]);
    pin(w1), pin(w5), pin(w8), pin(e3), pin(e6), pin(e7);
    const C g6 = lane_value(gth, 6), g7 = lane_value(gth, 7), g8 = lane_value(gth, 8);
    const C g15 = lane_value(gth, 15), g16 = lane_value(gth, 16), g17 = lane_value(gth, 17);
    const bool first = lane == 0, lastl = lane == G.last;
    f[0] = pass<kCopy>(raw[0]);
    f[2] = pass<kCopy>(raw[2]);
    f[4] = pass<kCopy>(raw[4]);
    f[1] = first ? g6 : w1;
    f[5] = first ? g7 : w5;
    f[8] = first ? g8 : w8;
    f[3] = lastl ? g15 : e3;
    f[6] = lastl ? g16 : e6;
    f[7] = lastl ? g17 : e7;
    rho = sum9(f);
    C h[9];
    h[0] = lane_value(gth, 0);
    h[2] = lane_value(gth, 1);
    h[4] = lane_value(gth, 2);
    h[1] = lane_value(gth, 3);
    h[5] = lane_value(gth, 4);
    h[8] = lane_value(gth, 5);
    h[3] = lane_value(raw[3], 0);
    h[6] = lane_value(raw[6], 0);
    h[7] = lane_value(raw[7], 0);
    rhoL = sum9(h);
    h[0] = lane_value(gth, 9);
    h[2] = lane_value(gth, 10);
    h[4] = lane_value(gth, 11);
    h[3] = lane_value(gth, 12);
    h[6] = lane_value(gth, 13);
    h[7] = lane_value(gth, 14);
    h[1] = lane_value(raw[1], G.last);
    h[5] = lane_value(raw[5], G.last);
    h[8] = lane_value(raw[8], G.last);
    rhoR = sum9(h);
}

template <bool kCopy, typename C>
__device__ inline void finish_g(const Strip& G, const C* raw, C gth, C* g) {
    const int lane = threadIdx.x & 63;
    C w1 = dpp_from_west(raw[1]), w5 = dpp_from_west(raw[5]), w8 = dpp_from_west(raw[8]);
    C e3 = dpp_from_east(raw[3]), e6 = dpp_from_east(raw[6]), e7 = dpp_from_east(raw[7]);
    pin(w1), pin(w5), pin(w8), pin(e3), pin(e6), pin(e7);
    const C g0 = lane_value(gth, 0), g1 = lane_value(gth, 1), g2 = lane_value(gth, 2);
    const C g3 = lane_value(gth, 3), g4 = lane_value(gth, 4), g5 = lane_value(gth, 5);
    const bool first = lane == 0, lastl = lane == G.last;
    g[0] = pass<kCopy>(raw[0]);
    g[2] = pass<kCopy>(raw[2]);
    g[4] = pass<kCopy>(raw[4]);
    g[1] = first ? g0 : w1;
    g[5] = first ? g1 : w5;
    g[8] = first ? g2 : w8;
    g[3] = lastl ? g3 : e3;
    g[6] = lastl ? g4 : e6;
    g[7] = lastl ? g5 : e7;
}

template <typename C>
struct Dens {
    C v, L, R;  // the lane's density and the two halo columns' densities (uniform)
};

// One row of the marching update.  kStage = 2: issue the loads for later rows (g of row
// y+2 into lg, f of row y+3 into lf), collide row y (f in fa, g in ga), store, then
// rotate the densities and finish the loads issued one row earlier: f of row y+2 from
// rf into fa (free once row y is collided; row y+1 sits in the caller's other array)
// and g of row y+1 from rg into ga; kStage = 1: the same without new loads; kStage = 0:
// collide and store only (last row).  The caller swaps the roles of the load targets
// and the finish sources every row, so no register holding a load in flight is copied.
// R[0..3] hold the byte offsets of rows y+1 .. y+4 (periodic); yo that of row y.
template <int kStage, typename S, typename C, bool kBuf, bool kSR>
__device__ __forceinline__ void ab_row(const Consts<C>& P, const Planes<S, kBuf>& in, const Planes<S, kBuf>& out,
                                       const Strip& G, typename OffT<kBuf>::type yo,
                                       const typename OffT<kBuf>::type (&R)[4], C (&fa)[9], const C (&rf)[9],
                                       const C& rfh, C (&lf)[9], C& lfh, C (&ga)[9], const C (&rg)[9],
                                       const C& rgh, C (&lg)[9], C& lgh, Dens<C>& dm, Dens<C>& dc, Dens<C>& dp) {
    constexpr bool kCopy = sizeof(S) >= 4;  // pass-through copies (see pass())
    const int lane = threadIdx.x & 63;
    if (kStage == 2) {
        load_target_row<S, C, kBuf>(in, 9, G, R[2], R[1], R[0], false, P.ref_g, lg, lgh);
        load_target_row<S, C, kBuf>(in, 0, G, R[3], R[2], R[1], true, P.ref_f, lf, lfh);
    }
    // neighbour densities: lane L-1 is x-1 (west), lane L+1 is x+1 (east); the
    // shifts run on the whole wavefront before the halo lanes are patched
    C wc = dpp_from_west(dc.v), ec = dpp_from_east(dc.v);
    C wm = dpp_from_west(dm.v), em = dpp_from_east(dm.v);
    C wp = dpp_from_west(dp.v), ep = dpp_from_east(dp.v);
    pin(wc), pin(ec), pin(wm), pin(em), pin(wp), pin(ep);
    const bool first = lane == 0, lastl = lane == G.last;
    const C rW = first ? dc.L : wc, rE = lastl ? dc.R : ec;
    const C rSW = first ? dm.L : wm, rSE = lastl ? dm.R : em;
    const C rNW = first ? dp.L : wp, rNE = lastl ? dp.R : ep;
    C sx, sy;
    stencil(rE, dp.v, rW, dm.v, rNE, rNW, rSW, rSE, sx, sy);
    C fo[9], go[9];
    collide(P, fa, ga, dc.v, sx, sy, fo, go);
    const typename OffT<kBuf>::type o = yo + G.xc * G.esz;
    if constexpr (kSR && sizeof(S) == 2) {
        // the random words of the two-column form: hash of the column pair, salt by
        // slot and by the column's place in the pair
        const bool odd = (G.xc & 1u) != 0;
        const uint32_t h = sr_node(yo + (G.xc & ~1u) * G.esz, G.srkey);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            out.template st_sr<C>(i, o, fo[i], P.ref_f[i], h ^ (odd ? kSrSalt.v[18 + i] : kSrSalt.v[i]), G.owner);
            out.template st_sr<C>(9 + i, o, go[i], P.ref_g[i], h ^ (odd ? kSrSalt.v[27 + i] : kSrSalt.v[9 + i]),
                                  G.owner);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            out.template st<C>(i, o, fo[i], P.ref_f[i], G.owner);
            out.template st<C>(9 + i, o, go[i], P.ref_g[i], G.owner);
        }
    }
    if (kStage >= 1) {
        dm = dc;
        dc = dp;
        finish_f<kCopy>(G, rf, rfh, fa, dp.v, dp.L, dp.R);
        finish_g<kCopy>(G, rg, rgh, ga);
    }
}

// Update of one work item (a strip of up to 64 columns times `rows` rows) of one
// lattice.  `w` must be uniform across the wavefront.
template <typename S, typename C, bool kBuf, bool kSR>
__device__ __forceinline__ void ab_strip(const S* __restrict__ in, S* __restrict__ out, const Consts<C>& P,
                                         const int w, const int nstrips, const int rows, const uint32_t step) {
    constexpr bool kCopy = sizeof(S) >= 4;  // pass-through copies (see pass())
    const int lane = threadIdx.x & 63;
    const int strip = w % nstrips, chunk = w / nstrips;
    const int nx = P.nx, ny = P.ny;
    const int x0 = strip * 64;
    const int owned = min(64, nx - x0);
    Strip G;
    G.nx = nx;
    G.ny = ny;
    G.rowb = (unsigned)nx * sizeof(S);
    G.esz = sizeof(S);
    G.owner = lane < owned;
    G.xc = (unsigned)(G.owner ? x0 + lane : nx - 1);
    G.last = __builtin_amdgcn_readfirstlane(owned - 1);  // a lane index for v_readlane: must be uniform
    G.srkey = kSR ? sr_key(step) : 0u;
    {
        // halo columns (uniform): x0-1, x0-2, x0+n, x0+n+1 modulo nx
        const unsigned l1 = __builtin_amdgcn_readfirstlane(wrap_row(x0 - 1, nx));
        const unsigned l2 = __builtin_amdgcn_readfirstlane(wrap_row(x0 - 2, nx));
        const unsigned r1 = __builtin_amdgcn_readfirstlane(wrap_row(x0 + owned, nx));
        const unsigned r2 = __builtin_amdgcn_readfirstlane(wrap_row(x0 + owned + 1, nx));
        // f slots (lane: population, column): 0-2 axis pops {0,2,4} at l1; 3-5 east pops
        // {1,5,8} at l2; 6-8 east pops at l1; 9-11 axis pops at r1; 12-14 west pops
        // {3,6,7} at r2; 15-17 west pops at r1.  g slots: 0-2 east pops at l1; 3-5 west
        // pops at r1.  Branch-free selects keep the setup free of divergent control flow.
        const int k = lane % 3, grp = lane / 3;
        const int axis0 = k == 0 ? 0 : (k == 1 ? 2 : 4);
        const int east = k == 0 ? 1 : (k == 1 ? 5 : 8);
        const int west = k == 0 ? 3 : (k == 1 ? 6 : 7);
        const int pf = (grp == 0 || grp == 3) ? axis0 : ((grp == 1 || grp == 2) ? east : west);
        const unsigned cf = grp == 1 ? l2 : (grp == 4 ? r2 : ((grp == 0 || grp == 2) ? l1 : r1));
        G.fon = lane < 18;
        G.fplane = (unsigned)pf;
        G.fcol = cf;
        G.fdy = pf == 2 || pf == 5 || pf == 6 ? -1 : (pf == 4 || pf == 7 || pf == 8 ? 1 : 0);  // -e_y
        const int pg = grp == 0 ? east : west;
        G.gon = lane < 6;
        G.gplane = (unsigned)pg;
        G.gcol = grp == 0 ? l1 : r1;
        G.gdy = pg == 5 || pg == 6 ? -1 : (pg == 7 || pg == 8 ? 1 : 0);
    }
    using Off = typename OffT<kBuf>::type;
    const size_t total = (size_t)18 * nx * ny * sizeof(S);
    const Planes<S, kBuf> Pin(in, total, G.rowb);
    const Planes<S, kBuf> Pout(out, total, G.rowb);
    const int y0 = chunk * rows, y1 = min(ny, y0 + rows);
    const Off blk = (Off)18 * G.rowb;  // bytes of one row block (all 18 slots of a row)
    const Off tot = (Off)total;

    // f of two consecutive rows in X and Y, g of the current row in gA; raw loads in
    // flight in C/D (f) and G/H (g), whose roles swap every row; densities of rows
    // y-1, y, y+1
    C fX[9], fY[9], gA[9], rC[9], hC, rD[9], hD, rG[9], hG, rH[9], hH;
    Dens<C> dm, dc, dp;
    // byte offsets of the row blocks of rows y0-2 .. y0+3 (periodic)
    Off ro[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int yy = __builtin_amdgcn_readfirstlane(wrap_row(y0 - 2 + k, ny));
        ro[k] = (Off)yy * blk;
    }
    {
        // all six prologue rows in flight at once (60 loads): one memory round trip
        // instead of one per row
        C r0[9], h0, r1[9], h1, r2[9], h2, r3[9], h3, t[9];
        load_target_row<S, C, kBuf>(Pin, 0, G, ro[2], ro[1], ro[0], true, P.ref_f, r0, h0);   // f(y0-1)
        load_target_row<S, C, kBuf>(Pin, 0, G, ro[3], ro[2], ro[1], true, P.ref_f, r1, h1);   // f(y0)
        load_target_row<S, C, kBuf>(Pin, 0, G, ro[4], ro[3], ro[2], true, P.ref_f, r2, h2);   // f(y0+1)
        load_target_row<S, C, kBuf>(Pin, 9, G, ro[3], ro[2], ro[1], false, P.ref_g, r3, h3);  // g(y0)
        load_target_row<S, C, kBuf>(Pin, 9, G, ro[4], ro[3], ro[2], false, P.ref_g, rG, hG);  // g(y0+1)
        load_target_row<S, C, kBuf>(Pin, 0, G, ro[5], ro[4], ro[3], true, P.ref_f, rC, hC);   // f(y0+2)
        finish_f<kCopy>(G, r0, h0, t, dm.v, dm.L, dm.R);
        finish_f<kCopy>(G, r1, h1, fX, dc.v, dc.L, dc.R);
        finish_f<kCopy>(G, r2, h2, fY, dp.v, dp.L, dp.R);
        finish_g<kCopy>(G, r3, h3, gA);
    }
    // Let the prologue's loads land before the loop: the loop header then sees only
    // the pipelined state, and the memory-counter waits inside the loop cover just the
    // loads issued in earlier rows (not the stores of the previous row).
#pragma unroll
    for (int i = 0; i < 9; ++i) asm volatile("" ::"v"(rG[i]), "v"(rC[i]));
    asm volatile("" ::"v"(hG), "v"(hC));
    Off R[4] = {ro[3], ro[4], ro[5], next_row<Off>(ro[5], blk, tot)};  // rows y+1 .. y+4
    Off yo = ro[2];
    auto advance = [&]() {
        yo = R[0];
        R[0] = R[1];
        R[1] = R[2];
        R[2] = R[3];
        R[3] = next_row<Off>(R[3], blk, tot);
    };
    int y = y0;
    for (; y < y1 - 3; y += 2) {
        ab_row<2, S, C, kBuf, kSR>(P, Pin, Pout, G, yo, R, fX, rC, hC, rD, hD, gA, rG, hG, rH, hH, dm, dc, dp);
        advance();
        ab_row<2, S, C, kBuf, kSR>(P, Pin, Pout, G, yo, R, fY, rD, hD, rC, hC, gA, rH, hH, rG, hG, dm, dc, dp);
        advance();
    }
    // ragged tail (once per strip): moves restore the roles the last rows expect
    if (y < y1 - 2) {
        ab_row<2, S, C, kBuf, kSR>(P, Pin, Pout, G, yo, R, fX, rC, hC, rD, hD, gA, rG, hG, rH, hH, dm, dc, dp);
        advance();
        ++y;
        // X now holds f(y+1) and Y f(y): swap them
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const C t = fX[i];
            fX[i] = fY[i];
            fY[i] = t;
            rC[i] = rD[i];
            rG[i] = rH[i];
        }
        hC = hD;
        hG = hH;
    }
    if (y < y1 - 1) {
        ab_row<1, S, C, kBuf, kSR>(P, Pin, Pout, G, yo, R, fX, rC, hC, rD, hD, gA, rG, hG, rH, hH, dm, dc, dp);
        yo = R[0];
        // the last row's f is in Y (X took f(y1), which no row collides)
#pragma unroll
        for (int i = 0; i < 9; ++i) fX[i] = fY[i];
    }
    ab_row<0, S, C, kBuf, kSR>(P, Pin, Pout, G, yo, R, fX, rC, hC, rD, hD, gA, rG, hG, rH, hH, dm, dc, dp);
}

template <typename S, typename C, int WPB, bool kBuf, bool kSR>
__global__ void __launch_bounds__(64 * WPB)
k_step_ab(const S* __restrict__ in, S* __restrict__ out, const Consts<C> P, const int nstrips,
          const int rows, const int nitems) {
    // the wavefront's work item is uniform across its lanes; saying so keeps the strip
    // geometry, the row loop and the halo columns on the scalar unit (and the loop free
    // of exec masking, which the DPP shifts rely on)
    const int w = __builtin_amdgcn_readfirstlane(remap_xcd(blockIdx.x, gridDim.x) * WPB + (int)(threadIdx.x >> 6));
    if (w >= nitems) return;
    ab_strip<S, C, kBuf, kSR>(in, out, P, w, nstrips, rows, P.step);
}

// ---------------------------------------------------------------------------
// fused two-buffer step, two columns per lane (128-column strips, even nx)
// ---------------------------------------------------------------------------
// Lane L holds the aligned column pair (x0 + 2L, x0 + 2L + 1): every row access is one
// 8-byte (FP32) or 4-byte (16-bit) load or store per lane, twice the bytes per
// instruction of the one-column form, and the pull shift needs one DPP per slot and
// pair: for e_x = +1 the first column takes the west lane's second value, for e_x = -1
// the second column takes the east lane's first value.  The gather slots, the halo
// columns and the order of every sum are those of the one-column form, so the result
// is bitwise the same.  Loads run two rows ahead: f of row y+3 and g of row y+2 are
// issued while row y collides (each row's arithmetic alone does not cover the memory
// latency at one or two wavefronts per SIMD).
template <typename S>
struct Bits2;
template <>
struct Bits2<float> {
    using V2 = unsigned __attribute__((ext_vector_type(2)));
    __device__ static void ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s, float& a, float& b) {
        // keep the builtin's own vector type: converting it to an ext_vector on
        // assignment compiles to a one-dword load whose value fills both elements
        const auto t = __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0);
        a = __builtin_bit_cast(float, (unsigned)t[0]);
        b = __builtin_bit_cast(float, (unsigned)t[1]);
    }
    __device__ static void st(float a, float b, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        V2 t;
        t.x = __builtin_bit_cast(unsigned, a);
        t.y = __builtin_bit_cast(unsigned, b);
        __builtin_amdgcn_raw_buffer_store_b64(t, r, v, s, kStreamStore);
    }
};
template <typename H>
struct Bits2Half {
    __device__ static void ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s, H& a, H& b) {
        const unsigned t = __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0);
        a = __builtin_bit_cast(H, (unsigned short)(t & 0xffffu));
        b = __builtin_bit_cast(H, (unsigned short)(t >> 16));
    }
    __device__ static void st(H a, H b, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        const unsigned t = (unsigned)__builtin_bit_cast(unsigned short, a) |
                           ((unsigned)__builtin_bit_cast(unsigned short, b) << 16);
        __builtin_amdgcn_raw_buffer_store_b32(t, r, v, s, kStreamStore);
    }
    __device__ static unsigned ldw(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0);
    }
    __device__ static void stw(unsigned t, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
        __builtin_amdgcn_raw_buffer_store_b32(t, r, v, s, kStreamStore);
    }
};
template <>
struct Bits2<__half> : Bits2Half<__half> {};
template <>
struct Bits2<__hip_bfloat16> : Bits2Half<__hip_bfloat16> {};

// Conversions of one 32-bit word holding a pair of 16-bit deviations (first column in
// the low half) with a uniform reference.  They give bitwise the same values as the
// per-value conversions of Io: FP16 to FP32 is exact, so f32(h) + ref and the fused
// h * 1 + ref round alike; the FP16 stores round once as in f16_dev; BF16 rounds to
// nearest even per value in both.
template <typename S>
struct Pair16;
template <>
struct Pair16<__half> {
    __device__ static void unpack(unsigned w, float ref, float& a, float& b) {
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(a) : "v"(w), "s"(ref));
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(b) : "v"(w), "s"(ref));
    }
    __device__ static unsigned pack(float a, float b, float ref) {
        unsigned t;
        asm("v_fma_mixlo_f16 %0, %1, 1.0, -%2" : "=v"(t) : "v"(a), "s"(ref));
        asm("v_fma_mixhi_f16 %0, %1, 1.0, -%2" : "+v"(t) : "v"(b), "s"(ref));
        return t;
    }
};
template <>
struct Pair16<__hip_bfloat16> {
    __device__ static void unpack(unsigned w, float ref, float& a, float& b) {
        a = __builtin_bit_cast(float, w << 16) + ref;
        b = __builtin_bit_cast(float, w & 0xffff0000u) + ref;
    }
    __device__ static unsigned pack(float a, float b, float ref) {
        using F2 = float __attribute__((ext_vector_type(2)));
        using B2 = __bf16 __attribute__((ext_vector_type(2)));
        const F2 v = {a - ref, b - ref};
        return __builtin_bit_cast(unsigned, __builtin_convertvector(v, B2));
    }
};

// pair access on top of Planes: slot i, byte offset of the pair's first column
// For 16-bit storage the pair stays packed in a (b is unused) until the row is
// finished (unpack2): converting right after the load would make the wavefront wait
// for the load there.
template <typename S, typename C>
__device__ inline void ld2(const Planes<S, true>& B, int i, unsigned off, C ref, C& a, C& b) {
    if constexpr (sizeof(S) == 2) {
        a = __builtin_bit_cast(C, Bits2<S>::ldw(B.r, off, B.ps * (unsigned)i));
        b = C(0);
    } else {
        S u, v;
        Bits2<S>::ld(B.r, off, B.ps * (unsigned)i, u, v);
        a = Io<S, C>::ld(&u, 0, ref);
        b = Io<S, C>::ld(&v, 0, ref);
    }
}
template <typename S, typename C>
__device__ inline void ld2(const Planes<S, false>& B, int i, size_t off, C ref, C& a, C& b) {
    if constexpr (sizeof(S) == 2) {
        a = __builtin_bit_cast(C, *reinterpret_cast<const unsigned*>(B.base + B.ps * i + off));
        b = C(0);
    } else {
        const S* q = reinterpret_cast<const S*>(B.base + B.ps * i + off);
        a = Io<S, C>::ld(q, 0, ref);
        b = Io<S, C>::ld(q, 1, ref);
    }
}

// Speed class of direction i (rest, axis, diagonal) as the index of the class's first
// direction: the 16-bit deviation references are class-uniform (set so on the host),
// and reading one entry per class keeps 6 instead of 18 of them live.
__device__ constexpr int kCls[9] = {0, 1, 1, 1, 1, 5, 5, 5, 5};

// Values of a finished row from the raw pair loads: 16-bit storage unpacks the words
// kept by ld2, wider storage takes the loaded values as they are.
template <typename S, typename C>
__device__ inline void unpack2(const C* ra, const C* rb, const C* ref, C* a, C* b) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if constexpr (sizeof(S) == 2) {
            Pair16<S>::unpack(__builtin_bit_cast(unsigned, ra[i]), ref[kCls[i]], a[i], b[i]);
        } else {
            a[i] = ra[i];
            b[i] = rb[i];
        }
    }
}
template <typename S, typename C>
__device__ inline void st2(const Planes<S, true>& B, int i, unsigned off, C a, C b, C ref, bool valid) {
    if constexpr (sizeof(S) == 2) {
        Bits2<S>::stw(Pair16<S>::pack(a, b, ref), B.r, valid ? off : B.drop, B.ps * (unsigned)i);
    } else {
        S u, v;
        Io<S, C>::st(&u, 0, a, ref);
        Io<S, C>::st(&v, 0, b, ref);
        Bits2<S>::st(u, v, B.r, valid ? off : B.drop, B.ps * (unsigned)i);
    }
}
template <typename S, typename C>
__device__ inline void st2(const Planes<S, false>& B, int i, size_t off, C a, C b, C ref, bool valid) {
    if (!valid) return;
    S* q = reinterpret_cast<S*>(B.base + B.ps * i + off);
    stream_store(q, a, ref);
    stream_store(q + 1, b, ref);
}
// 16-bit pair, stochastic rounding with the random words ra, rb
template <typename S, typename C>
__device__ inline void st2_sr(const Planes<S, true>& B, int i, unsigned off, C a, C b, C ref, uint32_t ra,
                              uint32_t rb, bool valid) {
    Bits2<S>::stw(Sr16<S>::pack(a, b, ref, ra, rb), B.r, valid ? off : B.drop, B.ps * (unsigned)i);
}
template <typename S, typename C>
__device__ inline void st2_sr(const Planes<S, false>& B, int i, size_t off, C a, C b, C ref, uint32_t ra,
                              uint32_t rb, bool valid) {
    if (valid)  // the pair's first column is even: a 4-byte aligned word
        __builtin_nontemporal_store(Sr16<S>::pack(a, b, ref, ra, rb), reinterpret_cast<unsigned*>(B.base + B.ps * i + off));
}

// Raw loads of one target row for both columns of the lane, and the gather.
template <typename S, typename C, bool kBuf>
__device__ inline void load_target_row2(const Planes<S, kBuf>& B, int first, const Strip& G,
                                        typename OffT<kBuf>::type up, typename OffT<kBuf>::type mid,
                                        typename OffT<kBuf>::type dn, bool is_f, const C* ref, C* ra, C* rb, C& gth) {
    using Off = typename OffT<kBuf>::type;
    const unsigned xo = G.xc * G.esz;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const Off r = kEy[i] < 0 ? up : (kEy[i] > 0 ? dn : mid);
        ld2<S, C>(B, first + i, r + xo, ref[i], ra[i], rb[i]);
    }
    const unsigned plane = is_f ? G.fplane : G.gplane;
    const unsigned col = is_f ? G.fcol : G.gcol;
    const int dy = is_f ? G.fdy : G.gdy;
    const bool on = is_f ? G.fon : G.gon;
    const Off r = dy > 0 ? up : (dy < 0 ? dn : mid);
    if constexpr (sizeof(S) == 2)
        gth = B.template gather_raw<C>(first + plane, r + col * G.esz, on);
    else
        gth = B.template gather<C>(first + plane, r + col * G.esz, on, ref[plane]);
}

// The gathered value of a finished row: 16-bit storage converts the bits kept by
// gather_raw with the reference of the lane's gather slot (a disabled slot read zero
// bits, as the converting gather does).
template <typename S, typename C>
__device__ inline C unpack_gather(C gth, C ref) {
    if constexpr (sizeof(S) == 2) {
        const S v = __builtin_bit_cast(S, (unsigned short)__builtin_bit_cast(unsigned, gth));
        return Io<S, C>::ld(&v, 0, ref);
    } else {
        return gth;
    }
}

template <typename C>
struct Dens2 {
    C a, b, L, R;  // the lane's two densities and the two halo columns' densities (uniform)
};

template <typename S, typename C>
__device__ inline void finish_f2(const Strip& G, const C* rawa, const C* rawb, C rawg, const C* ref, C* fa, C* fb,
                                 Dens2<C>& d) {
    constexpr bool kCopy = sizeof(S) >= 4;
    C ra[9], rb[9];
    unpack2<S>(rawa, rawb, ref, ra, rb);
    const C gth = unpack_gather<S>(rawg, C(G.fref));
    const int lane = threadIdx.x & 63;
    C w1 = dpp_from_west(rb[1]), w5 = dpp_from_west(rb[5]), w8 = dpp_from_west(rb[8]);
    C e3 = dpp_from_east(ra[3]), e6 = dpp_from_east(ra[6]), e7 = dpp_from_east(ra[7]);
    pin(w1), pin(w5), pin(w8), pin(e3), pin(e6), pin(e7);
    const C g6 = lane_value(gth, 6), g7 = lane_value(gth, 7), g8 = lane_value(gth, 8);
    const C g15 = lane_value(gth, 15), g16 = lane_value(gth, 16), g17 = lane_value(gth, 17);
    const bool first = lane == 0, lastl = lane == G.last;
    fa[0] = pass<kCopy>(ra[0]), fa[2] = pass<kCopy>(ra[2]), fa[4] = pass<kCopy>(ra[4]);
    fb[0] = pass<kCopy>(rb[0]), fb[2] = pass<kCopy>(rb[2]), fb[4] = pass<kCopy>(rb[4]);
    fa[1] = first ? g6 : w1, fb[1] = pass<kCopy>(ra[1]);
    fa[5] = first ? g7 : w5, fb[5] = pass<kCopy>(ra[5]);
    fa[8] = first ? g8 : w8, fb[8] = pass<kCopy>(ra[8]);
    fa[3] = pass<kCopy>(rb[3]), fb[3] = lastl ? g15 : e3;
    fa[6] = pass<kCopy>(rb[6]), fb[6] = lastl ? g16 : e6;
    fa[7] = pass<kCopy>(rb[7]), fb[7] = lastl ? g17 : e7;
    d.a = sum9(fa);
    d.b = sum9(fb);
    C h[9];
    h[0] = lane_value(gth, 0);
    h[2] = lane_value(gth, 1);
    h[4] = lane_value(gth, 2);
    h[1] = lane_value(gth, 3);
    h[5] = lane_value(gth, 4);
    h[8] = lane_value(gth, 5);
    h[3] = lane_value(ra[3], 0);
    h[6] = lane_value(ra[6], 0);
    h[7] = lane_value(ra[7], 0);
    d.L = sum9(h);
    h[0] = lane_value(gth, 9);
    h[2] = lane_value(gth, 10);
    h[4] = lane_value(gth, 11);
    h[3] = lane_value(gth, 12);
    h[6] = lane_value(gth, 13);
    h[7] = lane_value(gth, 14);
    h[1] = lane_value(rb[1], G.last);
    h[5] = lane_value(rb[5], G.last);
    h[8] = lane_value(rb[8], G.last);
    d.R = sum9(h);
}

template <typename S, typename C>
__device__ inline void finish_g2(const Strip& G, const C* rawa, const C* rawb, C rawg, const C* ref, C* ga, C* gb) {
    constexpr bool kCopy = sizeof(S) >= 4;
    C ra[9], rb[9];
    unpack2<S>(rawa, rawb, ref, ra, rb);
    const C gth = unpack_gather<S>(rawg, C(G.gref));
    const int lane = threadIdx.x & 63;
    C w1 = dpp_from_west(rb[1]), w5 = dpp_from_west(rb[5]), w8 = dpp_from_west(rb[8]);
    C e3 = dpp_from_east(ra[3]), e6 = dpp_from_east(ra[6]), e7 = dpp_from_east(ra[7]);
    pin(w1), pin(w5), pin(w8), pin(e3), pin(e6), pin(e7);
    const C g0 = lane_value(gth, 0), g1 = lane_value(gth, 1), g2 = lane_value(gth, 2);
    const C g3 = lane_value(gth, 3), g4 = lane_value(gth, 4), g5 = lane_value(gth, 5);
    const bool first = lane == 0, lastl = lane == G.last;
    ga[0] = pass<kCopy>(ra[0]), ga[2] = pass<kCopy>(ra[2]), ga[4] = pass<kCopy>(ra[4]);
    gb[0] = pass<kCopy>(rb[0]), gb[2] = pass<kCopy>(rb[2]), gb[4] = pass<kCopy>(rb[4]);
    ga[1] = first ? g0 : w1, gb[1] = pass<kCopy>(ra[1]);
    ga[5] = first ? g1 : w5, gb[5] = pass<kCopy>(ra[5]);
    ga[8] = first ? g2 : w8, gb[8] = pass<kCopy>(ra[8]);
    ga[3] = pass<kCopy>(rb[3]), gb[3] = lastl ? g3 : e3;
    ga[6] = pass<kCopy>(rb[6]), gb[6] = lastl ? g4 : e6;
    ga[7] = pass<kCopy>(rb[7]), gb[7] = lastl ? g5 : e7;
}

// One row of the two-column march.  kStage = 2: issue the raw loads of f(y+3) into lf and
// of g(y+2) into lg, collide row y (f in fa/fb, g in ga/gb) for both columns, store, then
// rotate the densities and finish the raw loads issued one row earlier: f(y+2) from rf
// into fa/fb (free once row y is collided; row y+1 sits in the caller's other pair) and
// g(y+1) from rg into ga/gb; kStage = 1: the same without new loads; kStage = 0: collide
// and store only (last row).  The load targets and the finish sources are separate
// arrays and the caller swaps their roles every row, so no register holding a load in
// flight is ever copied: a copy would stall the wavefront until that load lands.
// R[0..3]: byte offsets of the row blocks of rows y+1 .. y+4; yo: row y.
template <int kStage, typename S, typename C, bool kBuf, bool kSR>
__device__ __forceinline__ void ab_row2(const Consts<C>& P, const Planes<S, kBuf>& in, const Planes<S, kBuf>& out,
                                        const Strip& G, typename OffT<kBuf>::type yo,
                                        const typename OffT<kBuf>::type (&R)[4], C (&fa)[9], C (&fb)[9],
                                        const C (&rfa)[9], const C (&rfb)[9], const C& rfh, C (&lfa)[9],
                                        C (&lfb)[9], C& lfh, C (&ga)[9], C (&gb)[9], const C (&rga)[9],
                                        const C (&rgb)[9], const C& rgh, C (&lga)[9], C (&lgb)[9], C& lgh,
                                        Dens2<C>& dm, Dens2<C>& dc, Dens2<C>& dp) {
    const int lane = threadIdx.x & 63;
    if (kStage == 2) {
        load_target_row2<S, C, kBuf>(in, 9, G, R[2], R[1], R[0], false, P.ref_g, lga, lgb, lgh);  // g(y+2)
        load_target_row2<S, C, kBuf>(in, 0, G, R[3], R[2], R[1], true, P.ref_f, lfa, lfb, lfh);   // f(y+3)
    }
    C wc = dpp_from_west(dc.b), ec = dpp_from_east(dc.a);
    C wm = dpp_from_west(dm.b), em = dpp_from_east(dm.a);
    C wp = dpp_from_west(dp.b), ep = dpp_from_east(dp.a);
    pin(wc), pin(ec), pin(wm), pin(em), pin(wp), pin(ep);
    const bool first = lane == 0, lastl = lane == G.last;
    C sxa, sya, sxb, syb;
    // column a: west neighbour from the west lane (or the halo), east is column b
    stencil(dc.b, dp.a, first ? dc.L : wc, dm.a, dp.b, first ? dp.L : wp, first ? dm.L : wm, dm.b, sxa, sya);
    // column b: west is column a, east neighbour from the east lane (or the halo)
    stencil(lastl ? dc.R : ec, dp.b, dc.a, dm.b, lastl ? dp.R : ep, dp.a, dm.a, lastl ? dm.R : em, sxb, syb);
    const typename OffT<kBuf>::type o = yo + G.xc * G.esz;
    {
        C foa[9], goa[9], fob[9], gob[9];
        collide(P, fa, ga, dc.a, sxa, sya, foa, goa);
        collide(P, fb, gb, dc.b, sxb, syb, fob, gob);
        if constexpr (kSR && sizeof(S) == 2) {
            const uint32_t h = sr_node(o, G.srkey);  // G.xc is the pair's (even) first column
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                st2_sr<S, C>(out, i, o, foa[i], fob[i], P.ref_f[kCls[i]], h ^ kSrSalt.v[i], h ^ kSrSalt.v[18 + i],
                             G.owner);
                st2_sr<S, C>(out, 9 + i, o, goa[i], gob[i], P.ref_g[kCls[i]], h ^ kSrSalt.v[9 + i],
                             h ^ kSrSalt.v[27 + i], G.owner);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                st2<S, C>(out, i, o, foa[i], fob[i], P.ref_f[kCls[i]], G.owner);
                st2<S, C>(out, 9 + i, o, goa[i], gob[i], P.ref_g[kCls[i]], G.owner);
            }
        }
    }
    if (kStage >= 1) {
        dm = dc;
        dc = dp;
        finish_f2<S>(G, rfa, rfb, rfh, P.ref_f, fa, fb, dp);
        finish_g2<S>(G, rga, rgb, rgh, P.ref_g, ga, gb);
    }
}

// One work item of the two-column form: a strip of up to 128 columns (nx even).
template <typename S, typename C, bool kBuf, bool kSR>
__device__ __forceinline__ void ab_strip2(const S* __restrict__ in, S* __restrict__ out, const Consts<C>& P,
                                          const int w, const int nstrips, const int rows, const uint32_t step) {
    using Off = typename OffT<kBuf>::type;
    const int lane = threadIdx.x & 63;
    const int strip = w % nstrips, chunk = w / nstrips;
    const int nx = P.nx, ny = P.ny;
    const int x0 = strip * 128;
    const int owned = min(128, nx - x0);  // even
    Strip G;
    G.nx = nx;
    G.ny = ny;
    G.rowb = (unsigned)nx * sizeof(S);
    G.esz = sizeof(S);
    G.owner = 2 * lane < owned;
    G.xc = (unsigned)(G.owner ? x0 + 2 * lane : nx - 2);  // first column of the lane's pair
    G.last = __builtin_amdgcn_readfirstlane(owned / 2 - 1);
    G.srkey = kSR ? sr_key(step) : 0u;
    {
        const unsigned l1 = __builtin_amdgcn_readfirstlane(wrap_row(x0 - 1, nx));
        const unsigned l2 = __builtin_amdgcn_readfirstlane(wrap_row(x0 - 2, nx));
        const unsigned r1 = __builtin_amdgcn_readfirstlane(wrap_row(x0 + owned, nx));
        const unsigned r2 = __builtin_amdgcn_readfirstlane(wrap_row(x0 + owned + 1, nx));
        const int k = lane % 3, grp = lane / 3;
        const int axis0 = k == 0 ? 0 : (k == 1 ? 2 : 4);
        const int east = k == 0 ? 1 : (k == 1 ? 5 : 8);
        const int west = k == 0 ? 3 : (k == 1 ? 6 : 7);
        const int pf = (grp == 0 || grp == 3) ? axis0 : ((grp == 1 || grp == 2) ? east : west);
        const unsigned cf = grp == 1 ? l2 : (grp == 4 ? r2 : ((grp == 0 || grp == 2) ? l1 : r1));
        G.fon = lane < 18;
        G.fplane = (unsigned)pf;
        G.fcol = cf;
        G.fdy = pf == 2 || pf == 5 || pf == 6 ? -1 : (pf == 4 || pf == 7 || pf == 8 ? 1 : 0);
        const int pg = grp == 0 ? east : west;
        G.gon = lane < 6;
        G.gplane = (unsigned)pg;
        G.gcol = grp == 0 ? l1 : r1;
        G.gdy = pg == 5 || pg == 6 ? -1 : (pg == 7 || pg == 8 ? 1 : 0);
    }
    if constexpr (sizeof(S) == 2) {
        G.fref = pick9(P.ref_f, G.fplane);
        G.gref = pick9(P.ref_g, G.gplane);
    }
    const size_t total = (size_t)18 * nx * ny * sizeof(S);
    const Planes<S, kBuf> Pin(in, total, G.rowb);
    const Planes<S, kBuf> Pout(out, total, G.rowb);
    const int y0 = chunk * rows, y1 = min(ny, y0 + rows);
    const Off blk = (Off)18 * G.rowb;
    const Off tot = (Off)total;
    Off ro[6];  // row blocks of rows y0-2 .. y0+3
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int yy = __builtin_amdgcn_readfirstlane(wrap_row(y0 - 2 + k, ny));
        ro[k] = (Off)yy * blk;
    }
    // f of two consecutive rows in the pairs X and Y, g of the current row in gA; raw
    // loads in flight in C/D (f) and G/H (g), whose roles swap every row
    C fXa[9], fXb[9], fYa[9], fYb[9], gAa[9], gAb[9];
    C rCa[9], rCb[9], hC, rDa[9], rDb[9], hD, rGa[9], rGb[9], hG, rHa[9], rHb[9], hH;
    Dens2<C> dm, dc, dp;
    {
        // all six prologue rows in flight at once (60 loads): one memory round trip
        // instead of one per row
        C a0[9], b0[9], h0, a1[9], b1[9], h1, a2[9], b2[9], h2, a3[9], b3[9], h3, ta[9], tb[9];
        load_target_row2<S, C, kBuf>(Pin, 0, G, ro[2], ro[1], ro[0], true, P.ref_f, a0, b0, h0);   // f(y0-1)
        load_target_row2<S, C, kBuf>(Pin, 0, G, ro[3], ro[2], ro[1], true, P.ref_f, a1, b1, h1);   // f(y0)
        load_target_row2<S, C, kBuf>(Pin, 0, G, ro[4], ro[3], ro[2], true, P.ref_f, a2, b2, h2);   // f(y0+1)
        load_target_row2<S, C, kBuf>(Pin, 9, G, ro[3], ro[2], ro[1], false, P.ref_g, a3, b3, h3);  // g(y0)
        load_target_row2<S, C, kBuf>(Pin, 9, G, ro[4], ro[3], ro[2], false, P.ref_g, rGa, rGb, hG);  // g(y0+1)
        load_target_row2<S, C, kBuf>(Pin, 0, G, ro[5], ro[4], ro[3], true, P.ref_f, rCa, rCb, hC);   // f(y0+2)
        finish_f2<S>(G, a0, b0, h0, P.ref_f, ta, tb, dm);
        finish_f2<S>(G, a1, b1, h1, P.ref_f, fXa, fXb, dc);
        finish_f2<S>(G, a2, b2, h2, P.ref_f, fYa, fYb, dp);
        finish_g2<S>(G, a3, b3, h3, P.ref_g, gAa, gAb);
    }
    // let the prologue's loads land before the loop (as in the one-column form)
#pragma unroll
    for (int i = 0; i < 9; ++i) asm volatile("" ::"v"(rGa[i]), "v"(rGb[i]), "v"(rCa[i]), "v"(rCb[i]));
    asm volatile("" ::"v"(hG), "v"(hC));
    Off R[4] = {ro[3], ro[4], ro[5], next_row<Off>(ro[5], blk, tot)};  // rows y+1 .. y+4
    Off yo = ro[2];
    auto advance = [&]() {
        yo = R[0];
        R[0] = R[1];
        R[1] = R[2];
        R[2] = R[3];
        R[3] = next_row<Off>(R[3], blk, tot);
    };
    int y = y0;
    for (; y < y1 - 3; y += 2) {
        ab_row2<2, S, C, kBuf, kSR>(P, Pin, Pout, G, yo, R, fXa, fXb, rCa, rCb, hC, rDa, rDb, hD, gAa, gAb, rGa, rGb, hG,
                               rHa, rHb, hH, dm, dc, dp);
        advance();
        ab_row2<2, S, C, kBuf, kSR>(P, Pin, Pout, G, yo, R, fYa, fYb, rDa, rDb, hD, rCa, rCb, hC, gAa, gAb, rHa, rHb, hH,
                               rGa, rGb, hG, dm, dc, dp);
        advance();
    }
    // ragged tail (once per strip): moves restore the roles the last rows expect
    if (y < y1 - 2) {
        ab_row2<2, S, C, kBuf, kSR>(P, Pin, Pout, G, yo, R, fXa, fXb, rCa, rCb, hC, rDa, rDb, hD, gAa, gAb, rGa, rGb, hG,
                               rHa, rHb, hH, dm, dc, dp);
        advance();
        ++y;
        // X now holds f(y+1) and Y f(y): swap them
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const C ta = fXa[i], tb = fXb[i];
            fXa[i] = fYa[i];
            fXb[i] = fYb[i];
            fYa[i] = ta;
            fYb[i] = tb;
            rCa[i] = rDa[i];
            rCb[i] = rDb[i];
            rGa[i] = rHa[i];
            rGb[i] = rHb[i];
        }
        hC = hD;
        hG = hH;
    }
    if (y < y1 - 1) {
        ab_row2<1, S, C, kBuf, kSR>(P, Pin, Pout, G, yo, R, fXa, fXb, rCa, rCb, hC, rDa, rDb, hD, gAa, gAb, rGa, rGb, hG,
                               rHa, rHb, hH, dm, dc, dp);
        yo = R[0];
        // the last row's f is in Y (X took f(y1), which no row collides)
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            fXa[i] = fYa[i];
            fXb[i] = fYb[i];
        }
    }
    ab_row2<0, S, C, kBuf, kSR>(P, Pin, Pout, G, yo, R, fXa, fXb, rCa, rCb, hC, rDa, rDb, hD, gAa, gAb, rGa, rGb, hG, rHa,
                           rHb, hH, dm, dc, dp);
}

template <typename S, typename C, int WPB, bool kBuf, bool kSR>
__global__ void __launch_bounds__(64 * WPB)
k_step_ab2(const S* __restrict__ in, S* __restrict__ out, const Consts<C> P, const int nstrips, const int rows,
           const int nitems) {
    const int w = __builtin_amdgcn_readfirstlane(remap_xcd(blockIdx.x, gridDim.x) * WPB + (int)(threadIdx.x >> 6));
    if (w >= nitems) return;
    ab_strip2<S, C, kBuf, kSR>(in, out, P, w, nstrips, rows, P.step);
}

// ---------------------------------------------------------------------------
// batched form: many independent lattices, one launch per step
// ---------------------------------------------------------------------------
// The lattice owning global item w is found by a binary search over `starts` (uniform,
// so it runs on the scalar unit); its constants and buffers come from its descriptor.
// Grid mode: one wavefront per item, XCD-remapped as in the single-lattice kernel.
// Queue mode: a persistent grid; the item range is cut into `groups` contiguous
// ranges, one per XCD (a block's XCD is its index modulo 8), and the wavefronts of
// an XCD take items of its range from an atomic counter until it is exhausted.
// Every lattice must satisfy the 32-bit buffer-offset bound ((18 ny + 17) nx sizeof(S)
// + 64 < 2^32, checked on the host).
template <typename S, typename C, bool kSR>
__device__ __forceinline__ void batch_item(const BatchDesc<C>* __restrict__ desc, const int32_t* __restrict__ starts,
                                           uint32_t* __restrict__ steps, const int nlat, const int w,
                                           const int parity) {
    int lo = 0, hi = nlat - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    const int b = __builtin_amdgcn_readfirstlane(lo);
    const BatchDesc<C>* D = desc + b;
    const S* in = static_cast<const S*>(D->buf[parity]);
    S* out = const_cast<S*>(static_cast<const S*>(D->buf[parity ^ 1]));
    const int item = __builtin_amdgcn_readfirstlane(w - starts[b]);
    // the lattice's step count: this launch reads the parity-p counter; the wavefront of
    // the lattice's first item writes the count of the next launch into the other one
    // (read by nobody in this launch), with a vector store
    const uint32_t step = steps[2 * b + parity];
    if (item == 0 && (threadIdx.x & 63) == 0) steps[2 * b + (parity ^ 1)] = step + 1u;
    if constexpr (sizeof(S) <= 4) {
        if (D->cols == 2) {
            ab_strip2<S, C, true, kSR>(in, out, D->P, item, D->nstrips, D->rows, step);
            return;
        }
    }
    ab_strip<S, C, true, kSR>(in, out, D->P, item, D->nstrips, D->rows, step);
}

template <typename S, typename C, int WPB, bool kQueue, bool kSR>
__global__ void __launch_bounds__(64 * WPB)
k_step_ab_batch(const BatchDesc<C>* __restrict__ desc, const int32_t* __restrict__ starts,
                unsigned* __restrict__ queue, uint32_t* __restrict__ steps, const int nlat, const int nitems,
                const int parity, const int groups) {
    if (!kQueue) {
        const int w = __builtin_amdgcn_readfirstlane(remap_xcd(blockIdx.x, gridDim.x) * WPB + (int)(threadIdx.x >> 6));
        if (w >= nitems) return;
        batch_item<S, C, kSR>(desc, starts, steps, nlat, w, parity);
        return;
    }
    // counters of the other parity were used by the previous launch (complete by stream
    // order) and are next used by the following launch (after this one completes)
    if (blockIdx.x == 0 && threadIdx.x < 8) queue[(parity ^ 1) * 8 + threadIdx.x] = 0u;
    const int g = (int)(blockIdx.x % (unsigned)groups);
    const int lo = (int)(((long long)nitems * g) / groups);
    const int hi = (int)(((long long)nitems * (g + 1)) / groups);
    unsigned* ctr = queue + parity * 8 + g;
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned t = 0;
        if (lane == 0) t = atomicAdd(ctr, 1u);
        const int w = lo + (int)__builtin_amdgcn_readfirstlane(t);
        if (w >= hi) break;
        batch_item<S, C, kSR>(desc, starts, steps, nlat, w, parity);
    }
}

// ---------------------------------------------------------------------------
// AA pattern (one buffer, in place).  Even step: node x reads slot i of x and
// writes its post-collision f_i to slot opp(i) of x.  Odd step: node x reads
// slot opp(i) of x - e_i and writes slot i of x + e_i.  Each node's read set
// equals its write set, so the update is race-free in place; the density
// stencil reads a separate array written by k_density beforehand.
// ---------------------------------------------------------------------------
template <typename S, typename C>
__device__ inline void aa_offsets(int parity, int x, int y, int nx, int ny, int* rd_slot, int* rd_off,
                                  int* wr_slot, int* wr_off) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (parity == 0) {
            rd_slot[i] = i;
            rd_off[i] = y * nx + x;
            wr_slot[i] = kOpp[i];
            wr_off[i] = rd_off[i];
        } else {
            rd_slot[i] = kOpp[i];
            rd_off[i] = wrap(y - kEy[i], ny) * nx + wrap(x - kEx[i], nx);
            wr_slot[i] = i;
            wr_off[i] = wrap(y + kEy[i], ny) * nx + wrap(x + kEx[i], nx);
        }
    }
}

template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_step_aa(S* __restrict__ st, const double* __restrict__ rho_arr, const Consts<C> P, const int parity) {
    using IO = Io<S, C>;
    const int nx = P.nx, ny = P.ny;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    int rs[9], ro[9], ws[9], wo[9];
    aa_offsets<S, C>(parity, x, y, nx, ny, rs, ro, ws, wo);
    // node offsets k = y' nx + x' -> element index of slot s: k + (17 y' + s) nx
    C f[9], g[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const size_t b = (size_t)ro[i] + (size_t)(17 * (ro[i] / nx)) * nx;
        f[i] = IO::ld(st + b + (size_t)rs[i] * nx, 0, P.ref_f[i]);
        g[i] = IO::ld(st + b + (size_t)(9 + rs[i]) * nx, 0, P.ref_g[i]);
    }
    const int xe = wrap(x + 1, nx), xw = wrap(x - 1, nx);
    const int yn = wrap(y + 1, ny) * nx, ys = wrap(y - 1, ny) * nx, yc = y * nx;
    const C rho = (C)rho_arr[yc + x];
    C sx, sy;
    stencil((C)rho_arr[yc + xe], (C)rho_arr[yn + x], (C)rho_arr[yc + xw], (C)rho_arr[ys + x],
            (C)rho_arr[yn + xe], (C)rho_arr[yn + xw], (C)rho_arr[ys + xw], (C)rho_arr[ys + xe], sx, sy);
    C fo[9], go[9];
    collide(P, f, g, rho, sx, sy, fo, go);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const size_t b = (size_t)wo[i] + (size_t)(17 * (wo[i] / nx)) * nx;
        IO::st(st + b + (size_t)ws[i] * nx, 0, fo[i], P.ref_f[i]);
        IO::st(st + b + (size_t)(9 + ws[i]) * nx, 0, go[i], P.ref_g[i]);
    }
}

// Populations of node (x, y) at the current time.  layout 0: AA even parity (slot i
// at x); 1: AA odd parity (slot opp(i) at x - e_i); 2: the two-buffer scheme's pull
// convention (slot i at x - e_i).
template <typename S, typename C>
__device__ inline void load_node(const S* st, const Consts<C>& P, int layout, int x, int y, C* f, C* g) {
    using IO = Io<S, C>;
    const int nx = P.nx, ny = P.ny;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int slot = i, xs = x, ys = y;
        if (layout != 0) {
            slot = layout == 1 ? kOpp[i] : i;
            xs = wrap(x - kEx[i], nx);
            ys = wrap(y - kEy[i], ny);
        }
        f[i] = IO::ld(st + slot_index(slot, xs, ys, nx), 0, P.ref_f[i]);
        g[i] = IO::ld(st + slot_index(9 + slot, xs, ys, nx), 0, P.ref_g[i]);
    }
}

// Equilibrium state from macroscopic fields.  layout 0 (AA even parity) stores f_i(x)
// in slot i at x; layout 2 (two-buffer pull convention) stores it at x - e_i, where
// the first step's pull read finds it.
template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_init(S* __restrict__ st, const double* __restrict__ rho_in, const double* __restrict__ ux_in,
       const double* __restrict__ uy_in, const double* __restrict__ T_in, const Consts<C> P, const int layout) {
    using IO = Io<S, C>;
    const int N = P.nx * P.ny;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    const C rho = (C)rho_in[k], u = (C)ux_in[k], v = (C)uy_in[k], T = (C)T_in[k];
    const C ux = u * P.inv_c, uy = v * P.inv_c;
    const C pbe = p_be(P, rho, T);
    const C eta = pbe * P.inv_cs2 - rho;
    const C ru2 = rho * (ux * ux + uy * uy);
    C m[9], f[9];
    m[0] = rho;
    m[1] = C(-2) * rho + C(2) * eta + C(3) * ru2;
    m[2] = rho + P.beta * eta - C(3) * ru2;
    m[3] = rho * ux;
    m[4] = -rho * ux;
    m[5] = rho * uy;
    m[6] = -rho * uy;
    m[7] = rho * (ux * ux - uy * uy);
    m[8] = rho * ux * uy;
    from_moments(m, f);
    const C rek = rho * (P.cv * T + C(0.5) * (u * u + v * v));
    const C rhk = rek + pbe;
    C n[9], g[9];
    n[0] = rek;
    n[1] = C(-4) * rek + P.g1C * T;
    n[2] = C(4) * rek - P.g2C * T;
    n[3] = rhk * ux;
    n[4] = -rhk * ux;
    n[5] = rhk * uy;
    n[6] = -rhk * uy;
    n[7] = C(0);
    n[8] = C(0);
    from_moments(n, g);
    const int y = k / P.nx, x = k - y * P.nx;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int xs = layout == 2 ? wrap(x - kEx[i], P.nx) : x;
        const int ys = layout == 2 ? wrap(y - kEy[i], P.ny) : y;
        IO::st(st + slot_index(i, xs, ys, P.nx), 0, f[i], P.ref_f[i]);
        IO::st(st + slot_index(9 + i, xs, ys, P.nx), 0, g[i], P.ref_g[i]);
    }
}

template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_density(const S* __restrict__ st, const Consts<C> P, const int parity, double* __restrict__ rho) {
    const int N = P.nx * P.ny;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    const int y = k / P.nx, x = k - y * P.nx;
    C f[9], g[9];
    load_node(st, P, parity, x, y, f, g);
    rho[k] = (double)(f[0] + ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8])));
}

template <typename C>
__device__ inline void neighbour_sums(const double* rho, const Consts<C>& P, int x, int y, C& sx, C& sy,
                                      C& wsum) {
    const int nx = P.nx, ny = P.ny;
    const int xe = wrap(x + 1, nx), xw = wrap(x - 1, nx);
    const int yn = wrap(y + 1, ny) * nx, ys = wrap(y - 1, ny) * nx, yc = y * nx;
    const C rE = (C)rho[yc + xe], rN = (C)rho[yn + x], rW = (C)rho[yc + xw], rS = (C)rho[ys + x];
    const C rNE = (C)rho[yn + xe], rNW = (C)rho[yn + xw], rSW = (C)rho[ys + xw], rSE = (C)rho[ys + xe];
    stencil(rE, rN, rW, rS, rNE, rNW, rSW, rSE, sx, sy);
    wsum = (C(1) / C(3)) * ((rE + rN) + (rW + rS)) + (C(1) / C(12)) * ((rNE + rNW) + (rSW + rSE));
}

template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_moments(const S* __restrict__ st, const Consts<C> P, const int parity, const double* __restrict__ rho,
          double* __restrict__ ux, double* __restrict__ uy, double* __restrict__ T) {
    const int N = P.nx * P.ny;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    const int y = k / P.nx, x = k - y * P.nx;
    C f[9], g[9], m[9], n[9];
    load_node(st, P, parity, x, y, f, g);
    to_moments(f, m);
    to_moments(g, n);
    C sx, sy, ws;
    neighbour_sums(rho, P, x, y, sx, sy, ws);
    const Macro<C> M = macros(P, (C)rho[k], m[3], m[5], n[0], sx, sy);
    if (ux) ux[k] = (double)(P.c * M.uxh);
    if (uy) uy[k] = (double)(P.c * M.uyh);
    if (T) T[k] = (double)M.T;
}

// Per-block FP64 partial sums of the 8 diagnostics, in a fixed order.
template <typename S, typename C>
__global__ void __launch_bounds__(256)
k_invariants(const S* __restrict__ st, const Consts<C> P, const int parity, const double* __restrict__ rho,
             double* __restrict__ partials) {
    const int N = P.nx * P.ny;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = blockIdx.x * 256 + threadIdx.x; k < N; k += gridDim.x * 256) {
        const int y = k / P.nx, x = k - y * P.nx;
        C f[9], g[9], m[9], n[9];
        load_node(st, P, parity, x, y, f, g);
        to_moments(f, m);
        to_moments(g, n);
        C sx, sy, ws;
        neighbour_sums(rho, P, x, y, sx, sy, ws);
        const C r = (C)rho[k];
        const Macro<C> M = macros(P, r, m[3], m[5], n[0], sx, sy);
        double mass = 0, sg = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            mass += (double)f[i];
            sg += (double)g[i];
        }
        acc[0] += mass;
        acc[1] += (double)P.c * (double)m[3];
        acc[2] += (double)P.c * (double)m[5];
        acc[3] += sg;
        acc[4] += (double)P.dt * (double)M.q;
        acc[5] += (double)P.Ep_pre * ((double)r * (double)r / 6.0 + 0.5 * (double)r * (double)ws);
        acc[6] += (double)M.rho_ek;
        bool bad = !(r > C(0)) || !(M.T > C(0)) || !isfinite((double)M.T) || !isfinite((double)M.rho_ek);
        if (P.eos_kind == 0) bad = bad || !(P.bq * r < C(1));
        else bad = bad || !(P.bq * r < C(1));
        acc[7] += bad ? 1.0 : 0.0;
    }
    __shared__ double sm[8][256];
#pragma unroll
    for (int j = 0; j < 8; ++j) sm[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int j = 0; j < 8; ++j) sm[j][threadIdx.x] += sm[j][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < 8) partials[blockIdx.x * 8 + threadIdx.x] = sm[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_reduce_partials(const double* __restrict__ partials, int nblocks,
                                                         double* __restrict__ out) {
    __shared__ double sm[8][256];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] += partials[b * 8 + j];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) sm[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int j = 0; j < 8; ++j) sm[j][threadIdx.x] += sm[j][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < 8) out[threadIdx.x] = sm[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
bool generic_addressing() {
    const char* e = std::getenv("LBM_GENERIC_ADDRESSING");
    return e && e[0] == '1';
}

// The buffer-instruction path's offset bound (see Planes): every offset, including
// the drop offset plus a 16-byte access, stays below 2^32.
bool fits_32bit(int nx, int ny, size_t esz) {
    return ((size_t)18 * ny + 17) * (size_t)nx * esz + 64 < ((size_t)1 << 32);
}

template <typename S, typename C>
struct Launch {
    // the two-column form: 4- and 2-byte storage and an even row length
    static bool pair_columns(int nx) { return sizeof(S) <= 4 && nx % 2 == 0; }
    static hipError_t init(const void* cv, void* st, const double* r, const double* u, const double* v,
                           const double* T, int layout, hipStream_t s) {
        const Consts<C>& P = *static_cast<const Consts<C>*>(cv);
        const int N = P.nx * P.ny;
        hipLaunchKernelGGL((k_init<S, C>), dim3((N + 255) / 256), dim3(256), 0, s, static_cast<S*>(st), r,
                           u, v, T, P, layout);
        return hipGetLastError();
    }
    template <bool kBuf, bool kSR>
    static hipError_t step_ab_wpb(const S* i, S* o, const Consts<C>& P, int nstrips, int rows, int nitems, int wpb,
                                  int nblocks, hipStream_t s) {
        switch (wpb) {
            case 1: hipLaunchKernelGGL((k_step_ab<S, C, 1, kBuf, kSR>), dim3(nblocks), dim3(64), 0, s, i, o, P, nstrips, rows, nitems); break;
            case 2: hipLaunchKernelGGL((k_step_ab<S, C, 2, kBuf, kSR>), dim3(nblocks), dim3(128), 0, s, i, o, P, nstrips, rows, nitems); break;
            case 4: hipLaunchKernelGGL((k_step_ab<S, C, 4, kBuf, kSR>), dim3(nblocks), dim3(256), 0, s, i, o, P, nstrips, rows, nitems); break;
            case 8: hipLaunchKernelGGL((k_step_ab<S, C, 8, kBuf, kSR>), dim3(nblocks), dim3(512), 0, s, i, o, P, nstrips, rows, nitems); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    template <bool kBuf, bool kSR>
    static hipError_t step_ab2_wpb(const S* i, S* o, const Consts<C>& P, int nstrips, int rows, int nitems, int wpb,
                                   int nblocks, hipStream_t s) {
        switch (wpb) {
            case 1: hipLaunchKernelGGL((k_step_ab2<S, C, 1, kBuf, kSR>), dim3(nblocks), dim3(64), 0, s, i, o, P, nstrips, rows, nitems); break;
            case 2: hipLaunchKernelGGL((k_step_ab2<S, C, 2, kBuf, kSR>), dim3(nblocks), dim3(128), 0, s, i, o, P, nstrips, rows, nitems); break;
            case 4: hipLaunchKernelGGL((k_step_ab2<S, C, 4, kBuf, kSR>), dim3(nblocks), dim3(256), 0, s, i, o, P, nstrips, rows, nitems); break;
            case 8: hipLaunchKernelGGL((k_step_ab2<S, C, 8, kBuf, kSR>), dim3(nblocks), dim3(512), 0, s, i, o, P, nstrips, rows, nitems); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    static hipError_t step_ab(const void* cv, const void* in, void* out, LaunchShape sh, bool sr, hipStream_t s) {
        if constexpr (sizeof(S) == 2) {
            if (sr) return step_ab_sr<true>(cv, in, out, sh, s);
        }
        return step_ab_sr<false>(cv, in, out, sh, s);
    }
    template <bool kSR>
    static hipError_t step_ab_sr(const void* cv, const void* in, void* out, LaunchShape sh, hipStream_t s) {
        const Consts<C>& P = *static_cast<const Consts<C>*>(cv);
        if constexpr (sizeof(S) <= 4) {
            if (pair_columns(P.nx) && sh.columns_per_lane != 1) {
                const int nstrips = (P.nx + 127) / 128;
                const int rows = sh.rows_per_wave;
                const int nitems = nstrips * ((P.ny + rows - 1) / rows);
                const int wpb = sh.waves_per_block;
                const int nblocks = (nitems + wpb - 1) / wpb;
                const bool kBuf = fits_32bit(P.nx, P.ny, sizeof(S)) && !generic_addressing();
                const S* i = static_cast<const S*>(in);
                S* o = static_cast<S*>(out);
                if (kBuf) return step_ab2_wpb<true, kSR>(i, o, P, nstrips, rows, nitems, wpb, nblocks, s);
                return step_ab2_wpb<false, kSR>(i, o, P, nstrips, rows, nitems, wpb, nblocks, s);
            }
        }
        const int nstrips = (P.nx + 63) / 64;
        const int rows = sh.rows_per_wave;
        const int nchunks = (P.ny + rows - 1) / rows;
        const int nitems = nstrips * nchunks;
        const int wpb = sh.waves_per_block;
        const int nblocks = (nitems + wpb - 1) / wpb;
        const S* i = static_cast<const S*>(in);
        S* o = static_cast<S*>(out);
        // raw buffer addressing needs every offset and the drop offset in 32 bits;
        // LBM_GENERIC_ADDRESSING=1 selects the 64-bit path for any size (for tests)
        const bool kBuf = fits_32bit(P.nx, P.ny, sizeof(S)) && !generic_addressing();
        if (kBuf) return step_ab_wpb<true, kSR>(i, o, P, nstrips, rows, nitems, wpb, nblocks, s);
        return step_ab_wpb<false, kSR>(i, o, P, nstrips, rows, nitems, wpb, nblocks, s);
    }
    template <int WPB, bool kSR>
    static hipError_t batch_wpb(const void* d, const int32_t* st, unsigned* q, uint32_t* steps, int nlat, int nitems,
                                int parity, BatchLaunch bl, hipStream_t s) {
        const BatchDesc<C>* desc = static_cast<const BatchDesc<C>*>(d);
        if (bl.queue)
            hipLaunchKernelGGL((k_step_ab_batch<S, C, WPB, true, kSR>), dim3(bl.blocks), dim3(64 * WPB), 0, s, desc, st,
                               q, steps, nlat, nitems, parity, bl.groups);
        else
            hipLaunchKernelGGL((k_step_ab_batch<S, C, WPB, false, kSR>), dim3(bl.blocks), dim3(64 * WPB), 0, s, desc,
                               st, q, steps, nlat, nitems, parity, bl.groups);
        return hipGetLastError();
    }
    template <bool kSR>
    static hipError_t batch_sr(const void* d, const int32_t* st, unsigned* q, uint32_t* steps, int nlat, int nitems,
                               int parity, BatchLaunch bl, hipStream_t s) {
        switch (bl.waves_per_block) {
            case 1: return batch_wpb<1, kSR>(d, st, q, steps, nlat, nitems, parity, bl, s);
            case 2: return batch_wpb<2, kSR>(d, st, q, steps, nlat, nitems, parity, bl, s);
            case 4: return batch_wpb<4, kSR>(d, st, q, steps, nlat, nitems, parity, bl, s);
            default: return hipErrorInvalidValue;
        }
    }
    static hipError_t step_ab_batch(const void* d, const int32_t* st, unsigned* q, uint32_t* steps, int nlat,
                                    int nitems, int parity, BatchLaunch bl, bool sr, hipStream_t s) {
        if constexpr (sizeof(S) == 2) {
            if (sr) return batch_sr<true>(d, st, q, steps, nlat, nitems, parity, bl, s);
        }
        return batch_sr<false>(d, st, q, steps, nlat, nitems, parity, bl, s);
    }
    template <int WPB, bool kSR>
    static int occ_wpb(int queue) {
        int n = 0;
        hipError_t e = queue ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                   &n, reinterpret_cast<const void*>(&k_step_ab_batch<S, C, WPB, true, kSR>), 64 * WPB, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                   &n, reinterpret_cast<const void*>(&k_step_ab_batch<S, C, WPB, false, kSR>), 64 * WPB, 0);
        return e == hipSuccess ? n : 0;
    }
    template <bool kSR>
    static int occ_sr(int wpb, int queue) {
        switch (wpb) {
            case 1: return occ_wpb<1, kSR>(queue);
            case 2: return occ_wpb<2, kSR>(queue);
            case 4: return occ_wpb<4, kSR>(queue);
            default: return 0;
        }
    }
    static int batch_occupancy(int wpb, int queue, bool sr) {
        if constexpr (sizeof(S) == 2) {
            if (sr) return occ_sr<true>(wpb, queue);
        }
        return occ_sr<false>(wpb, queue);
    }
    static hipError_t step_aa(const void* cv, void* st, double* rho, int parity, LaunchShape, hipStream_t s) {
        const Consts<C>& P = *static_cast<const Consts<C>*>(cv);
        const int N = P.nx * P.ny;
        hipLaunchKernelGGL((k_density<S, C>), dim3((N + 255) / 256), dim3(256), 0, s,
                           static_cast<const S*>(st), P, parity, rho);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_step_aa<S, C>), dim3((P.nx + 63) / 64, (P.ny + 3) / 4), dim3(256), 0, s,
                           static_cast<S*>(st), rho, P, parity);
        return hipGetLastError();
    }
    static hipError_t density(const void* cv, const void* st, int parity, double* rho, hipStream_t s) {
        const Consts<C>& P = *static_cast<const Consts<C>*>(cv);
        const int N = P.nx * P.ny;
        hipLaunchKernelGGL((k_density<S, C>), dim3((N + 255) / 256), dim3(256), 0, s,
                           static_cast<const S*>(st), P, parity, rho);
        return hipGetLastError();
    }
    static hipError_t moments(const void* cv, const void* st, int parity, const double* rho, double* ux,
                              double* uy, double* T, hipStream_t s) {
        const Consts<C>& P = *static_cast<const Consts<C>*>(cv);
        const int N = P.nx * P.ny;
        hipLaunchKernelGGL((k_moments<S, C>), dim3((N + 255) / 256), dim3(256), 0, s,
                           static_cast<const S*>(st), P, parity, rho, ux, uy, T);
        return hipGetLastError();
    }
    static hipError_t invariants(const void* cv, const void* st, int parity, const double* rho,
                                 double* partials, double* result, hipStream_t s) {
        const Consts<C>& P = *static_cast<const Consts<C>*>(cv);
        const int N = P.nx * P.ny;
        int nb = (N + 255) / 256;
        if (nb > kMaxPartialBlocks) nb = kMaxPartialBlocks;
        hipLaunchKernelGGL((k_invariants<S, C>), dim3(nb), dim3(256), 0, s, static_cast<const S*>(st), P,
                           parity, rho, partials);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partials, nb, result);
        return hipGetLastError();
    }
};

}  // namespace

#define LBM_DISPATCH(prec, call)                                        \
    switch (prec) {                                                     \
        case kF64: return Launch<double, double>::call;                 \
        case kF32: return Launch<float, float>::call;                   \
        case kF16: return Launch<__half, float>::call;                  \
        case kBF16: return Launch<__hip_bfloat16, float>::call;         \
        default: return hipErrorInvalidValue;                           \
    }

hipError_t launch_init(int prec, const void* c, void* state, const double* rho, const double* ux,
                       const double* uy, const double* T, int layout, hipStream_t stream) {
    LBM_DISPATCH(prec, init(c, state, rho, ux, uy, T, layout, stream));
}
hipError_t launch_step_ab(int prec, const void* c, const void* in, void* out, LaunchShape shape, bool stochastic,
                          hipStream_t stream) {
    LBM_DISPATCH(prec, step_ab(c, in, out, shape, stochastic, stream));
}
hipError_t launch_step_aa(int prec, const void* c, void* state, double* rho_scratch, int parity,
                          LaunchShape shape, hipStream_t stream) {
    LBM_DISPATCH(prec, step_aa(c, state, rho_scratch, parity, shape, stream));
}
hipError_t launch_density(int prec, const void* c, const void* state, int aa_parity, double* rho,
                          hipStream_t stream) {
    LBM_DISPATCH(prec, density(c, state, aa_parity, rho, stream));
}
hipError_t launch_moments(int prec, const void* c, const void* state, int aa_parity, const double* rho,
                          double* ux, double* uy, double* T, hipStream_t stream) {
    LBM_DISPATCH(prec, moments(c, state, aa_parity, rho, ux, uy, T, stream));
}
hipError_t launch_invariants(int prec, const void* c, const void* state, int aa_parity, const double* rho,
                             double* partials, double* result, hipStream_t stream) {
    LBM_DISPATCH(prec, invariants(c, state, aa_parity, rho, partials, result, stream));
}

hipError_t launch_step_ab_batch(int prec, const void* desc, const int32_t* starts, unsigned* queue,
                                uint32_t* steps, int nlat, int nitems, int parity, BatchLaunch bl, bool stochastic,
                                hipStream_t stream) {
    LBM_DISPATCH(prec, step_ab_batch(desc, starts, queue, steps, nlat, nitems, parity, bl, stochastic, stream));
}
int batch_blocks_per_cu(int prec, int waves_per_block, int queue, bool stochastic) {
    switch (prec) {
        case kF64: return Launch<double, double>::batch_occupancy(waves_per_block, queue, false);
        case kF32: return Launch<float, float>::batch_occupancy(waves_per_block, queue, false);
        case kF16: return Launch<__half, float>::batch_occupancy(waves_per_block, queue, stochastic);
        case kBF16: return Launch<__hip_bfloat16, float>::batch_occupancy(waves_per_block, queue, stochastic);
        default: return 0;
    }
}
size_t batch_desc_size(int prec) { return prec == kF64 ? sizeof(BatchDesc<double>) : sizeof(BatchDesc<float>); }

size_t consts_size(int prec) { return prec == kF64 ? sizeof(Consts<double>) : sizeof(Consts<float>); }
size_t storage_bytes(int prec) { return prec == kF64 ? 8 : (prec == kF32 ? 4 : 2); }

}  // namespace lbm_dev
