#!/bin/bash
# Builds the library with AddressSanitizer and UBSan on its host code only
# (device code is compiled as usual), and the test program abi_sanitize.cpp that
# calls every C-ABI entry point, into tests/native/_build/.  Run the program
# on a machine with the GPU:
#   ASAN_OPTIONS=detect_leaks=0:halt_on_error=1 UBSAN_OPTIONS=halt_on_error=1 \
#     tests/native/_build/abi_sanitize
# (leak detection is off: the HIP runtime keeps its own allocations to the
# end of the process).
set -euo pipefail
here="$(cd "$(dirname "$0")" && pwd)"
repo="$(cd "$here/../.." && pwd)"
out="$here/_build"
mkdir -p "$out"
hipcc="${HIPCC:-/opt/rocm/bin/hipcc}"
"$hipcc" --offload-arch=gfx950 -O2 -g -std=c++20 -fPIC -shared -ffp-contract=on \
  -Xclang -target-feature -Xclang -packed-fp32-ops \
  -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer \
  -I "$repo/include" "$repo/paper_1301_3423_amd/csrc/rlb_capi.hip" -o "$out/librlb_asan.so"
"$hipcc" -O1 -g -std=c++17 -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined \
  -I "$repo/include" "$here/abi_sanitize.cpp" -L "$out" -lrlb_asan -Wl,-rpath,'$ORIGIN' -o "$out/abi_sanitize"
echo "built $out/abi_sanitize"
