// Constants of the DCT entropy code shared by its kernels and the C ABI.
#pragma once

namespace tomo {

constexpr int ECODE_INTERVAL = 64;     // blocks per restart interval
constexpr int ECODE_MAX_BITS = 2302;   // longest code of one block: DC 33 + 63 x (3 + 33) + 1 bits

}  // namespace tomo
