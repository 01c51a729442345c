#!/bin/bash
# Host-side sanitizer runs, on the CPU (no GPU is used):
#   1. the oracle built with AddressSanitizer + UndefinedBehaviorSanitizer
#      (gcc) under the CPU test suite;
#   2. the library's host code (plan builder, C ABI) built with
#      AddressSanitizer + UndefinedBehaviorSanitizer (clang, host pass only)
#      under the CPU test suite;
#   3. the threaded host plan builder built with ThreadSanitizer, through a
#      small driver that creates host-only plans.
# Usage: tests/sanitize/run_sanitizers.sh   (from anywhere; builds under
# _build_sanitize/ at the repository root)
set -euo pipefail
ROOT=$(cd "$(dirname "$0")/../.." && pwd)
OUT=$ROOT/_build_sanitize
CSRC=$ROOT/paper_2010_02857_amd/csrc
mkdir -p "$OUT"
HIPCC=/opt/rocm/bin/hipcc
CLANG_RT=$(ls -d /opt/rocm/llvm/lib/clang/*/lib/linux | head -1)
SRCS="plan.hip plan_gpu.hip kernels.hip api.hip"
GPUFLAGS="-O1 -g -std=c++17 -fPIC --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops"

echo "== oracle: ASan + UBSan (gcc)"
gcc -O1 -g -std=c11 -fopenmp -ffp-contract=off -fPIC -shared -fno-omit-frame-pointer \
    -fsanitize=address,undefined -fno-sanitize-recover=undefined \
    -o "$OUT/liboracle_asan.so" "$ROOT/oracle/ifgf_oracle.c" -lm
( cd "$ROOT" && LD_PRELOAD="$(gcc -print-file-name=libasan.so):$(gcc -print-file-name=libubsan.so)" \
  ASAN_OPTIONS=detect_leaks=0 IFGF_ORACLE_LIB="$OUT/liboracle_asan.so" OMP_NUM_THREADS=4 \
  python3 -m pytest tests/test_oracle.py -x -q -m "not gpu" -p no:cacheprovider )

echo "== library host code: ASan + UBSan (clang, host pass)"
objs=""
for s in $SRCS; do
    $HIPCC $GPUFLAGS -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined \
        -Xarch_host -fno-omit-frame-pointer -c "$CSRC/$s" -o "$OUT/asan_${s%.hip}.o"
    objs="$objs $OUT/asan_${s%.hip}.o"
done
$HIPCC --offload-arch=gfx950 -shared -fPIC -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined \
    -shared-libsan -o "$OUT/libifgf_asan.so" $objs -lpthread
( cd "$ROOT" && LD_PRELOAD="$CLANG_RT/libclang_rt.asan-x86_64.so" ASAN_OPTIONS=detect_leaks=0 \
  IFGF_LIB="$OUT/libifgf_asan.so" OMP_NUM_THREADS=4 \
  python3 -m pytest tests/test_abi.py -x -q -m "not gpu" -p no:cacheprovider )

echo "== host plan builder: TSan (clang, host pass)"
objs=""
for s in $SRCS; do
    $HIPCC $GPUFLAGS -Xarch_host -fsanitize=thread -c "$CSRC/$s" -o "$OUT/tsan_${s%.hip}.o"
    objs="$objs $OUT/tsan_${s%.hip}.o"
done
$HIPCC -O1 -g -std=c++17 -Xarch_host -fsanitize=thread -c "$ROOT/tests/sanitize/plan_driver.cpp" \
    -o "$OUT/tsan_driver.o"
$HIPCC --offload-arch=gfx950 -Xarch_host -fsanitize=thread -o "$OUT/plan_driver_tsan" $objs "$OUT/tsan_driver.o" \
    -lpthread
TSAN_OPTIONS="halt_on_error=1" IFGF_HOST_THREADS=8 "$OUT/plan_driver_tsan"
echo "== sanitizer runs clean"
