// Wave primitives the leaf executor's arithmetic is written against: lane
// masks (ballot), per-lane mask bits, reads of one lane's value, 32-bit limb
// operations with carry, funnel shifts and scheduling hints.  On gfx950 they
// are the amdgcn builtins.  When TFT_WAVE_EMU is defined (host test builds
// only) the same names come from a lockstep emulation of one wavefront that
// the including file provides before this header (namespace tft::lf2::emu).
#pragma once
#include <stdint.h>

#if defined(TFT_WAVE_EMU)

#define TFT_DINL inline

namespace tft {
namespace lf2 {
inline uint64_t ballot(bool p) { return emu::ballot(p); }
inline bool lane_bit(uint64_t m) { return ((m >> emu::lane()) & 1ull) != 0ull; }
inline uint32_t lane_id() { return emu::lane(); }
inline uint32_t uni(uint32_t v) { return emu::readlane(v, 0); }
inline uint32_t readlane(uint32_t v, int l) { return emu::readlane(v, l); }
inline uint32_t alignbit(uint32_t hi, uint32_t lo, uint32_t s) {
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> (s & 31u));
}
inline uint32_t opaque_zero() { return 0u; }
inline void opaque(uint32_t &) {}
// LDS words by byte address: the emulation's addresses are byte offsets from
// the start of the array
inline uint32_t lds_addr(const uint32_t *) { return 0u; }
inline uint32_t lds_word(const uint32_t *sm, uint32_t byte_addr) { return sm[byte_addr / 4u]; }
inline void sched_barrier() {}
// LDS written by some lanes and then read by others of the same wave: a
// wavefront executes each instruction for all lanes, the emulation has to wait
inline void wave_sync() { emu::sync(); }
inline uint32_t addc(uint32_t a, uint32_t b, uint32_t &c) {
    const uint64_t s = (uint64_t)a + b + c;
    c = (uint32_t)(s >> 32);
    return (uint32_t)s;
}
inline uint32_t subb(uint32_t a, uint32_t b, uint32_t &c) {
    const uint64_t s = (uint64_t)a - b - c;
    c = (uint32_t)(s >> 63);
    return (uint32_t)s;
}
}  // namespace lf2
}  // namespace tft

#else

#include <hip/hip_runtime.h>

#define TFT_DINL __device__ __forceinline__ __attribute__((always_inline))

namespace tft {
namespace lf2 {
TFT_DINL uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
TFT_DINL bool lane_bit(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }
TFT_DINL uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }
TFT_DINL uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
TFT_DINL uint32_t readlane(uint32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }
TFT_DINL uint32_t alignbit(uint32_t hi, uint32_t lo, uint32_t s) { return __builtin_amdgcn_alignbit(hi, lo, s); }
// a zero the compiler cannot see through: keeps x + 0 + carry a carry chain
TFT_DINL uint32_t opaque_zero() {
    uint32_t z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    return z;
}
// The value stays in its register and the compiler may not fold how it was
// computed into later instructions.  Placed after a limb chain whose last
// carry is dropped: otherwise the compiler merges that chain's last limb
// (x - borrow) into the next chain's first addition of the same limb as
// x + (-borrow) + carry, which has the right sum but the wrong carry out.
TFT_DINL void opaque(uint32_t &x) { asm volatile("" : "+v"(x)); }
// LDS words by byte address in the workgroup's LDS: an address chosen per lane
// at run time feeds a ds_read directly, with the word's constant offset in the
// instruction's immediate field.
typedef __attribute__((address_space(3))) const uint32_t lds_cu32;
TFT_DINL uint32_t lds_addr(const uint32_t *sm) {
    return (uint32_t)(uintptr_t)(lds_cu32 *)sm;
}
TFT_DINL uint32_t lds_word(const uint32_t *, uint32_t byte_addr) { return *(lds_cu32 *)(uintptr_t)byte_addr; }
TFT_DINL void sched_barrier() { __builtin_amdgcn_sched_barrier(0); }
// a wavefront runs every lane through each instruction in order: nothing to do
TFT_DINL void wave_sync() {}
TFT_DINL uint32_t addc(uint32_t a, uint32_t b, uint32_t &c) {
    uint32_t co;
    const uint32_t r = __builtin_addc(a, b, c, &co);
    c = co;
    return r;
}
TFT_DINL uint32_t subb(uint32_t a, uint32_t b, uint32_t &c) {
    uint32_t co;
    const uint32_t r = __builtin_subc(a, b, c, &co);
    c = co;
    return r;
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
}  // namespace lf2
}  // namespace tft

#endif
