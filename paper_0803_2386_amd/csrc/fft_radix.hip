// The level kernel k_pass (fft_pass.h) with register stages of radix 4, 8 or
// 32 instead of 16: the general-radix FFT of Ch. 1 ("Performance of the
// General-Radix FFT", Fig. radnbutterfly, Table 4), where the radix trades
// the number of passes through the fast memory level (here: LDS exchanges
// and barriers) against the work and registers of one butterfly.  Selected
// per level through the tuning block (complex64 levels of 2^5 .. 2^14 points
// that run the level kernel); radix 32 needs 32 points a thread (mode 1).
#include "fft_pass.h"

namespace moa {

namespace {

using PassFn = void (*)(PassArgs);

constexpr int kRadixLgnMin = 5;
constexpr int kRadixLgnMax = kMaxLgBlockC64;

#define MOA_RADIX_ROW(L, G)                                                                               \
    {                                                                                                     \
        {&k_pass<float, L, 0, false, false, G>, &k_pass<float, L, 0, false, true, G>,                   \
         &k_pass<float, L, 0, true, false, G>, &k_pass<float, L, 0, true, true, G>},                    \
            {&k_pass<float, L, 1, false, false, G>, nullptr, nullptr, &k_pass<float, L, 1, true, true, G>}, \
        {                                                                                                 \
            nullptr, &k_pass<float, L, 2, false, true, G>, &k_pass<float, L, 2, true, false, G>, nullptr   \
        }                                                                                                 \
    }
#define MOA_RADIX32_ROW(L) \
    {                      \
        {nullptr, nullptr, nullptr, nullptr}, {&k_pass<float, L, 1, false, false, 5>, nullptr, nullptr, &k_pass<float, L, 1, true, true, 5>}, \
        {                  \
            nullptr, nullptr, nullptr, nullptr \
        }                  \
    }
#define MOA_RADIX_TABLE(ROW) \
    { ROW(5), ROW(6), ROW(7), ROW(8), ROW(9), ROW(10), ROW(11), ROW(12), ROW(13), ROW(14) }
#define MOA_R4(L) MOA_RADIX_ROW(L, 2)
#define MOA_R8(L) MOA_RADIX_ROW(L, 3)

// [lgn - 5][mode][tin][tout]
static const PassFn kRadix4[kRadixLgnMax - kRadixLgnMin + 1][3][4] = MOA_RADIX_TABLE(MOA_R4);
static const PassFn kRadix8[kRadixLgnMax - kRadixLgnMin + 1][3][4] = MOA_RADIX_TABLE(MOA_R8);
static const PassFn kRadix32[kRadixLgnMax - kRadixLgnMin + 1][3][4] = MOA_RADIX_TABLE(MOA_RADIX32_ROW);

}  // namespace

const void* radix_pass_fn(const PassDesc& d)
{
    if (d.lgn < kRadixLgnMin || d.lgn > kRadixLgnMax || d.kmode < 0 || d.kmode > 2) return nullptr;
    const int col = (d.in_tile_fast ? 2 : 0) + (d.out_tile_fast ? 1 : 0);
    const int row = d.lgn - kRadixLgnMin;
    PassFn f = nullptr;
    if (d.lgrad == 2) f = kRadix4[row][d.kmode][col];
    else if (d.lgrad == 3) f = kRadix8[row][d.kmode][col];
    else if (d.lgrad == 5) f = kRadix32[row][d.kmode][col];
    return reinterpret_cast<const void*>(f);
}

}  // namespace moa
