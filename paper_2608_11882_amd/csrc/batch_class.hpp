#pragma once

// batch_class.hpp -- tile width classes of the batched sweeps (device
// constants shared by batch_kernels.hip and batch2_kernels.hip).

namespace hc {

// Width class c: 8 << c lanes per row, NT >> (3 + c) rows.  A class exists
// for a block size when it has at least 4 rows and one thread per ring
// element (with the four corners the two-step tile also stages).
template <int NT, int CLS>
struct WidthClass {
    static constexpr int lanes = 8 << CLS;
    static constexpr int rows = NT / lanes;
    static constexpr bool valid = rows >= 4 && NT >= 2 * lanes + 2 * rows + 4;
};

}  // namespace hc
