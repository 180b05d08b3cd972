// Radix-16 instantiations of the level kernel k_pass (fft_pass.h) and the
// dispatch of a pass descriptor to its kernel: the paired-column, short,
// matrix-core and other-radix kernels live in their own files.
#include "fft_pass.h"

namespace moa {

// ---------------------------------------------------------------------------
// Kernel table: [lgn][mode][tin][tout]; mode 1 exists for tin == tout only,
// mode 2 for tin != tout only, complex128 uses mode 0.
// ---------------------------------------------------------------------------
using PassFn = void (*)(PassArgs);

#define MOA_PASS_ROW32(L)                                                                                      \
    {                                                                                                          \
        {&k_pass<float, L, 0, false, false>, &k_pass<float, L, 0, false, true>, &k_pass<float, L, 0, true, false>, \
         &k_pass<float, L, 0, true, true>},                                                                    \
            {&k_pass<float, L, 1, false, false>, nullptr, nullptr, &k_pass<float, L, 1, true, true>},          \
        {                                                                                                      \
            nullptr, &k_pass<float, L, 2, false, true>, &k_pass<float, L, 2, true, false>, nullptr             \
        }                                                                                                      \
    }
#define MOA_PASS_MODES64(L) \
    { &k_pass<double, L, 0, false, false>, &k_pass<double, L, 0, false, true>, &k_pass<double, L, 0, true, false>, \
      &k_pass<double, L, 0, true, true> }

static const PassFn kPass32[kMaxLgBlockC64 + 1][3][4] = {
    MOA_PASS_ROW32(0),  MOA_PASS_ROW32(1),  MOA_PASS_ROW32(2),  MOA_PASS_ROW32(3),  MOA_PASS_ROW32(4),
    MOA_PASS_ROW32(5),  MOA_PASS_ROW32(6),  MOA_PASS_ROW32(7),  MOA_PASS_ROW32(8),  MOA_PASS_ROW32(9),
    MOA_PASS_ROW32(10), MOA_PASS_ROW32(11), MOA_PASS_ROW32(12), MOA_PASS_ROW32(13), MOA_PASS_ROW32(14)};

static const PassFn kPass64[kMaxLgBlockC128 + 1][4] = {
    MOA_PASS_MODES64(0),  MOA_PASS_MODES64(1),  MOA_PASS_MODES64(2),  MOA_PASS_MODES64(3),  MOA_PASS_MODES64(4),
    MOA_PASS_MODES64(5),  MOA_PASS_MODES64(6),  MOA_PASS_MODES64(7),  MOA_PASS_MODES64(8),  MOA_PASS_MODES64(9),
    MOA_PASS_MODES64(10), MOA_PASS_MODES64(11), MOA_PASS_MODES64(12), MOA_PASS_MODES64(13)};

static PassFn pass_fn_lookup(bool fp64, const PassDesc& d)
{
    const int lgn = d.lgn, km = d.kmode;
    const bool tin = d.in_tile_fast, tout = d.out_tile_fast;
    if (d.lgrad != 0 && d.lgrad != kLgRadix)
        return fp64 ? nullptr : reinterpret_cast<PassFn>(const_cast<void*>(radix_pass_fn(d)));
    const int mode = (tin ? 2 : 0) + (tout ? 1 : 0);
    if (lgn < 0 || km < 0 || km > 2) return nullptr;
    if (fp64) return (lgn <= kMaxLgBlockC128 && km == 0) ? kPass64[lgn][mode] : nullptr;
    return lgn <= kMaxLgBlockC64 ? kPass32[lgn][km][mode] : nullptr;
}

const void* pass_kernel_fn(bool fp64, const PassDesc& d, bool fwd)
{
    if (d.mfma) return mfma_kernel_fn(d, fwd);
    if (d.kmode == 3) return pair_kernel_fn(d, fwd);
    if (d.kmode == 4) return small_kernel_fn(fp64, d, fwd);
    return reinterpret_cast<const void*>(pass_fn_lookup(fp64, d));
}

hipError_t prepare_pass_kernel(bool fp64, const PassDesc& d)
{
    if (d.mfma) return prepare_mfma_kernel(d);
    if (d.kmode == 3) return prepare_pair_kernel(d);
    if (d.kmode == 4) return prepare_small_kernel(fp64, d);
    PassFn f = pass_fn_lookup(fp64, d);
    if (!f) return hipErrorInvalidValue;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(f), hipFuncAttributeMaxDynamicSharedMemorySize,
                               d.lds_bytes);
}

hipError_t launch_pass(bool fp64, const PassDesc& d, const PassArgs& a, hipStream_t s)
{
    if (d.mfma) return launch_mfma(d, a, s);
    if (d.kmode == 3) return launch_pair(d, a, s);
    if (d.kmode == 4) return launch_small(fp64, d, a, s);
    PassFn f = pass_fn_lookup(fp64, d);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(unsigned(d.grid)), dim3(unsigned(d.threads)), d.lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace moa
