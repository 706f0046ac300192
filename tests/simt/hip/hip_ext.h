#pragma once
#include "../simt.h"
